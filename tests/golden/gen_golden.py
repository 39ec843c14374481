"""Write tests/golden/oracle_vectors.txt from the CPU oracle alone.

Each line: length, the four key words, the message in hex ('-' if empty) and
the four words of the 256-bit hash (the 64- and 128-bit hashes are its first
one and two words).  Lengths cover 0..100, both sides of every packet
boundary up to 8 packets, and a few longer messages.  Run from the repo root:
    python tests/golden/gen_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402

SEED = 1612062570
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_vectors.txt")


def lengths():
    ls = list(range(0, 101))
    for k in range(4, 9):
        ls += [32 * k - 1, 32 * k, 32 * k + 1]
    ls += [32 * 9 + 9, 32 * 10 + 18, 32 * 11 + 27, 1000, 1024, 2047]
    return ls


def main():
    rng = np.random.Generator(np.random.PCG64(SEED))
    rows = []
    for L in lengths():
        key = rng.integers(0, 2**64, size=4, dtype=np.uint64)
        if L % 7 == 3:
            msg = np.zeros(L, np.uint8)  # some all-zero messages
        else:
            msg = np.frombuffer(rng.bytes(L), dtype=np.uint8)
        h = oracle.hash256(key, msg)
        rows.append("%d %s %s %s" % (L, " ".join("%016x" % int(k) for k in key),
                                     msg.tobytes().hex() or "-",
                                     " ".join("%016x" % x for x in h)))
    with open(OUT, "w") as f:
        f.write("# length key0 key1 key2 key3 message_hex h0 h1 h2 h3 (written by gen_golden.py from the oracle)\n")
        f.write("\n".join(rows) + "\n")


if __name__ == "__main__":
    main()
