"""Helpers for the GPU tests: move seeded batches to the device and compare
the HIP results with the oracle bit for bit."""
import sys

import numpy as np
import torch

import oracle

PATHS = ("lane1", "lane4", "bucketed", "auto")


def require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a visible AMD GPU")
    from paper_1612_06257_amd import hh
    hh.lib()  # fails loudly if libhh.so is missing
    return hh


def announce(*what):
    print("[gpu-case]", *what, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    a = np.ascontiguousarray(a)
    if not a.flags.writeable:  # e.g. np.frombuffer over bytes; torch wants writable memory
        a = a.copy()
    t = torch.from_numpy(a)
    if dtype is not None:
        t = t.view(dtype)
    return t.cuda()


def batch_to_device(keys, key_idx, data, offsets, lengths):
    k = dev(np.asarray(keys, np.uint64).reshape(-1, 4), torch.int64)
    d = dev(np.asarray(data, np.uint8)) if len(data) else torch.zeros(0, dtype=torch.uint8,
                                                                       device="cuda")
    o = dev(np.asarray(offsets, np.uint64), torch.int64)
    L = dev(np.asarray(lengths, np.uint64), torch.int64)
    ki = None if key_idx is None else dev(np.asarray(key_idx, np.uint32), torch.int32)
    return k, ki, d, o, L


def run(hh, path, width, keys, key_idx, data, offsets, lengths):
    k, ki, d, o, L = batch_to_device(keys, key_idx, data, offsets, lengths)
    out = hh.hash(k, d, o, L, ki, width=width, path=path)
    torch.cuda.synchronize()
    return hh.to_u64(out)


def oracle_ref(width, keys, key_idx, data, offsets, lengths):
    return oracle.batch(keys, key_idx, data, offsets, lengths, width)


def assert_same(got, want, ctx=""):
    got = np.asarray(got).reshape(want.shape)
    bad = np.nonzero(np.any(got != want, axis=1))[0]
    assert bad.size == 0, "%s: %d of %d messages differ, first at %s" % (
        ctx, bad.size, want.shape[0], bad[:8].tolist())
