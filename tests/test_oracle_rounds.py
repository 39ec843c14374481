"""Pin of the oracle's padding layout by the round-count study of Sec. 4.3.

Sec. 4.3 hashes all 2^24 three-byte inputs and reports, for the flip rate of
an output bit when one input bit flips: strong biases after two finalization
rounds, a drop by a factor of about 300 to 0.03% after three, and no
measurable change from a fourth.  Three-byte inputs go entirely through the
remainder step (Sec. 4.5), so the figures depend on where the padded packet
puts the last r%4 bytes; tests/golden/rounds_study_grid.md holds the study
for every reading of the padding text (written by gen_rounds_study.py).

The statistic: bias = |2p - 1| per (input bit, output bit) cell of the 64-bit
hash, averaged over the 24 x 64 cells, p counted over the 2^23 input pairs
differing in that bit.  A random function gives sqrt(2/pi)/sqrt(2^23), about
0.0276%, which is the paper's 0.03%.
"""
import math
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "hh_oracle.c")
DRIVER = os.path.join(HERE, "rounds_study_main.c")

# the key of the GPU rounds study
KEY = ("0123456789abcdef", "fedcba9876543210", "0f1e2d3c4b5a6978", "8877665544332211")
NULL_MEAN = math.sqrt(2 / math.pi) / math.sqrt(2 ** 23)


def round_biases(oracle_src, workdir, rounds=4, key=KEY, variant="oracle"):
    """{k: (mean bias, max bias)} after k = 1..rounds finalization rounds, for
    the oracle built from ``oracle_src``."""
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = os.path.join(str(workdir), "rounds_study")
    subprocess.run(["gcc", "-std=c99", "-O2", "-pthread", DRIVER, oracle_src, "-o", exe],
                   check=True, capture_output=True)
    threads = max(1, min(os.cpu_count() or 1, 16))
    out = subprocess.run([exe, *key, str(rounds), str(threads), variant], check=True,
                         capture_output=True, text=True, timeout=600).stdout
    res = {}
    for line in out.split("\n"):
        if line.strip():
            _, k, mean, mx = line.split()
            res[int(k)] = (float(mean), float(mx))
    return res


def check_rounds_figures(res):
    """Sec. 4.3's figures, as bounds on the mean bias."""
    b2, b3, b4 = res[2][0], res[3][0], res[4][0]
    assert b2 > 0.01, "two rounds should leave strong biases: %.4f%%" % (100 * b2)
    assert b2 / b3 > 100, "three rounds should cut the bias by two orders: %.1fx" % (b2 / b3)
    assert b3 < 2 * NULL_MEAN, "three rounds should reach about 0.03%%: %.4f%%" % (100 * b3)
    assert abs(b4 - NULL_MEAN) < 0.1 * NULL_MEAN, \
        "four rounds should sit at a random function's level: %.4f%%" % (100 * b4)


def test_oracle_reproduces_the_round_count_figures(tmp_path):
    check_rounds_figures(round_biases(SRC, tmp_path))


def test_former_layout_needs_a_fourth_round(tmp_path):
    # the study driver's reading "t28/L/64" (every r%4 tail at packet bytes
    # 28..) stays far above the random level after three rounds
    res = round_biases(SRC, tmp_path, variant="t28/L/64")
    assert res[3][0] > 4 * NULL_MEAN
    with pytest.raises(AssertionError):
        check_rounds_figures(res)
