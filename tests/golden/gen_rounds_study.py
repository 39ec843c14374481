"""Write tests/golden/rounds_study_grid.md: the finalization-round study of
Sec. 4.3 on the CPU, for the oracle and for every alternative reading of the
Sec. 4.5 padding text that the study driver knows (tests/rounds_study_main.c).

All 2^24 three-byte inputs under one key, rounds 1..5, mean and max over the
24 x 64 (input bit, output bit) cells of |2p - 1|.  Sec. 4.3 reports strong
biases after two rounds, a drop by a factor of about 300 to 0.03% after
three, and no measurable change from a fourth.  Run from the repo root
(about 2 minutes per key on 8 cores):
    python tests/golden/gen_rounds_study.py
"""
import math
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "rounds_study_grid.md")

# the key of the GPU rounds study, then three more
KEYS = [
    ("0123456789abcdef", "fedcba9876543210", "0f1e2d3c4b5a6978", "8877665544332211"),
    ("9e3779b97f4a7c15", "bf58476d1ce4e5b9", "94d049bb133111eb", "0000000000000000"),
    ("ffffffffffffffff", "ffffffffffffffff", "ffffffffffffffff", "ffffffffffffffff"),
    ("0000000000000001", "0000000000000002", "0000000000000003", "0000000000000004"),
]
FULL_GRID = (["oracle"] + ["%s/%s/%s" % (p, r, i) for p in ("t28", "t29", "half", "h13")
                           for r in "LR" for i in ("64", "32")]
             + ["t20/L/64", "t4/L/64", "cont/L/64"])
KEY_GRID = ["oracle", "t28/L/64", "half/L/64", "h13/L/64", "t20/L/64"]


def build(exe):
    cmd = ["gcc", "-std=c99", "-O2", "-pthread", os.path.join(ROOT, "tests", "rounds_study_main.c"),
           os.path.join(ROOT, "oracle", "hh_oracle.c"), "-o", exe]
    subprocess.run(cmd, check=True)


def run(exe, key, rounds, variants, threads):
    out = subprocess.run([exe, *key, str(rounds), str(threads), *variants], check=True,
                         capture_output=True, text=True).stdout
    rows = {}
    for line in out.split("\n"):
        if line.strip():
            name, k, mean, mx = line.split()
            rows.setdefault(name, {})[int(k)] = (float(mean), float(mx))
    return rows


def main():
    if shutil.which("gcc") is None:
        sys.exit("gcc not found")
    threads = min(os.cpu_count() or 1, 16)
    null = math.sqrt(2 / math.pi) / math.sqrt(2 ** 23)
    lines = [
        "# Finalization-round study (Sec. 4.3) under readings of the padding text (Sec. 4.5)",
        "",
        "Written by `tests/golden/gen_rounds_study.py` (CPU, oracle + `tests/rounds_study_main.c`).",
        "All 2^24 three-byte inputs under one key; cell (b, o) counts, over the 2^23 input pairs",
        "that differ in bit b, how often bit o of the 64-bit hash toggles; bias = |2p - 1|.",
        "Mean and max over the 24 x 64 cells, in percent.  A random function gives a mean",
        "of sqrt(2/pi)/sqrt(2^23) = %.4f%%." % (100 * null),
        "",
        "Placement of the last r%4 tail bytes (3-byte inputs: all three bytes):",
        "t28 = packet bytes 28.. (top dword of the packet); t29 = the packet's top bytes;",
        "half = top dword of the 16-byte half being filled (bytes 12.. for r < 16, 28.. for",
        "r >= 16); h13 = top bytes of that half; t20, t4 = top dword of lane 2 / lane 0;",
        "cont = right after the whole 4-byte groups.  Rotation of the v1 halves: L/R.",
        "Size injection: 64 = one 64-bit add of r*(2^32+1), 32 = two 32-bit adds.",
        "`oracle` is the oracle's own remainder step.",
        "",
    ]
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "rounds_study")
        build(exe)
        for n, key in enumerate(KEYS):
            variants = FULL_GRID if n == 0 else KEY_GRID
            rows = run(exe, key, 5, variants, threads)
            lines += ["## key %s" % " ".join(key), "",
                      "| reading | 1 round | 2 | 3 | 4 | 5 | 3-round max |",
                      "|---|---|---|---|---|---|---|"]
            for name in variants:
                r = rows[name]
                lines.append("| %s | %s | %.3f |" % (
                    name, " | ".join("%.4f" % (100 * r[k][0]) for k in range(1, 6)), 100 * r[3][1]))
            lines.append("")
            print("key %d done" % n, flush=True)
    with open(OUT, "w") as f:
        f.write("\n".join(lines))


if __name__ == "__main__":
    main()
