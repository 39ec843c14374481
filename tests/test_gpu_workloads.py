"""Parity at the full sizes of the four batch workloads, in the launch
configuration the benchmark times (GPU required).  Every message of every
workload is compared bit for bit with the oracle."""
import os

import numpy as np
import pytest

from _gpu import announce, assert_same, oracle_ref, require_gpu, run
from paper_1612_06257_amd import workloads as W

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def hh():
    return require_gpu()


def _check(hh, b, path, width):
    announce(b.name, path, "width", width)
    want = oracle_ref_threads(width, b)
    got = run(hh, path, width, b.keys, b.key_idx, b.data, b.offsets, b.lengths)
    assert_same(got, want, "%s %s w%d" % (b.name, path, width))


def oracle_ref_threads(width, b):
    import oracle
    return oracle.batch(b.keys, b.key_idx, b.data, b.offsets, b.lengths, width, n_threads=THREADS)


def test_plain_fixed_4096x1k(hh):
    b = W.plain_fixed()
    for path in ("auto", "lane1", "lane4"):
        _check(hh, b, path, 1)


def test_short_mixed_all_widths(hh):
    b = W.short_mixed()
    for width in (1, 2, 4):
        _check(hh, b, "auto", width)
    _check(hh, b, "lane1", 1)


def test_prf_counters_2e24(hh):
    b = W.prf_counters()
    _check(hh, b, "auto", 1)


def test_lognormal_2gib(hh):
    b = W.lognormal()
    _check(hh, b, "auto", 1)
