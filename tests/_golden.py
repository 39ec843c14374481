"""Reader for tests/golden/oracle_vectors.txt (written by gen_golden.py)."""
import os

import numpy as np

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_vectors.txt")


def load_vectors():
    """List of (key uint64[4], message uint8[L], hash256 list of 4 ints)."""
    out = []
    with open(PATH) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            L = int(t[0])
            key = np.array([int(x, 16) for x in t[1:5]], dtype=np.uint64)
            msg = np.frombuffer(bytes.fromhex(t[5]) if t[5] != "-" else b"", dtype=np.uint8)
            assert msg.size == L
            h = [int(x, 16) for x in t[6:10]]
            out.append((key, msg, h))
    return out
