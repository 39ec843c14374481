"""Avalanche studies on the GPU (needs the GPU).

    python -m paper_1612_06257_amd.avalanche smhasher [--samples N] [--trials T]
    python -m paper_1612_06257_amd.avalanche rounds

* smhasher (Sec. 6.1): for input sizes 4..32 bytes, N random (key, message)
  samples per trial, every single input-bit flip; the bias of a trial is the
  largest deviation of any (input bit, output bit) flip rate from 1/2, as
  abs(2p - 1); the reported value is the median over T trials.  The paper
  used 30M samples and 49 trials and reports medians of 0.064-0.076% for
  HighwayHash, SipHash and RDRAND alike.  Next to it: the median bias of a
  truly random function with the same number of cells and samples (drawn
  from binomial counts), the floor any good hash sits on.
* rounds (Sec. 4.3): all 2^24 three-byte inputs under one key, 1..4
  finalization rounds, max and mean bias per round count.  Each input and its
  flipped partner are both enumerated, so a cell's flip rate rests on 2^23
  distinct pairs; a random function's mean bias is sqrt(2/pi)/sqrt(2^23).

Inputs come from SplitMix64 (any strong generator stands in for the paper's
pcg64_k32; the kernel and the host implement it separately).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def bias_of(counts: np.ndarray, n: int):
    dev = np.abs(2.0 * counts / n - 1.0)
    return float(dev.max()), float(dev.mean())


def null_median_max_bias(cells: int, n: int, trials: int, seed: int = 1) -> float:
    rng = np.random.default_rng(seed)
    m = [np.abs(2.0 * rng.binomial(n, 0.5, size=cells) / n - 1.0).max() for _ in range(trials)]
    return float(np.median(m))


def smhasher(sizes, n: int, trials: int, seed: int = 2017):
    import torch
    from . import hh
    out = []
    for size in sizes:
        t0 = time.perf_counter()
        biases = []
        for t in range(trials):
            c = hh.avalanche_counts(size, n, 4, seed=seed + 1000 * size + t)
            biases.append(bias_of(c.cpu().numpy(), n)[0])
        torch.cuda.synchronize()
        rec = {"study": "avalanche", "size": size, "samples": n, "trials": trials,
               "median_bias_pct": 100 * float(np.median(biases)),
               "max_bias_pct": 100 * float(np.max(biases)),
               "null_median_bias_pct": 100 * null_median_max_bias(8 * size * 64, n, trials),
               "seconds": time.perf_counter() - t0}
        print(json.dumps(rec), flush=True)
        out.append(rec)
    return out


def rounds_study(key=(0x0123456789ABCDEF, 0xFEDCBA9876543210, 0x0F1E2D3C4B5A6978,
                      0x8877665544332211), msg_bytes: int = 3, rounds=(1, 2, 3, 4)):
    from . import hh
    n = 1 << (8 * msg_bytes)
    out = []
    for r in rounds:
        t0 = time.perf_counter()
        c = hh.avalanche_counts(msg_bytes, n, r, key=key).cpu().numpy()
        mx, mean = bias_of(c, n)
        rec = {"study": "rounds", "msg_bytes": msg_bytes, "inputs": n, "rounds": r,
               "max_bias_pct": 100 * mx, "mean_bias_pct": 100 * mean,
               "null_mean_bias_pct": 100 * float(np.sqrt(2 / np.pi) / np.sqrt(n // 2)),
               "seconds": time.perf_counter() - t0}
        print(json.dumps(rec), flush=True)
        out.append(rec)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["smhasher", "rounds"])
    ap.add_argument("--samples", type=int, default=30_000_000)
    ap.add_argument("--trials", type=int, default=49)
    ap.add_argument("--sizes", default="4-32")
    args = ap.parse_args(argv)
    if args.study == "rounds":
        rounds_study()
        return 0
    lo, _, hi = args.sizes.partition("-")
    sizes = range(int(lo), int(hi or lo) + 1)
    smhasher(sizes, args.samples, args.trials)
    return 0


if __name__ == "__main__":
    sys.exit(main())
