"""The serving loop on the GPU: every request's result in the mixed,
continuously batched run equals the same request hashed alone (one-shot
kernel) and the oracle, bit for bit; admission stays within the budget."""
import numpy as np
import pytest
import torch

import oracle
from _gpu import announce, require_gpu
from paper_1612_06257_amd import serve, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hh():
    return require_gpu()


@pytest.mark.parametrize("source", ["device", "host"])
def test_serving_results_match_alone_and_oracle(hh, source):
    announce("serving", source)
    tr = workloads.serving_trace(400, 20000.0, lo=1, hi=200000, n_keys=16, seed=99)
    tr.lengths[::23] = 0
    budget = 8 << 20
    backend = serve.GpuBackend(tr.keys, tr.data, budget, 256, source)
    srv = serve.Server(backend, budget_bytes=budget, chunk_bytes=4096)
    reqs = serve.requests_from_trace(tr)
    m = srv.run(reqs)
    assert m["completed"] == len(reqs)
    assert m["max_bytes_in_flight"] <= budget
    # alone: each request through the one-shot batched kernel, one message per call
    keys = torch.from_numpy(tr.keys).view(torch.int64).cuda()
    data = torch.from_numpy(tr.data).cuda()
    for r in reqs:
        msg = tr.data[r.src:r.src + r.length]
        want = tuple(oracle.hash_words(tr.keys[r.key_idx], msg, r.width))
        assert r.result == want, r.rid
    sample = reqs[::7]
    offs = torch.tensor([r.src for r in sample], dtype=torch.int64, device="cuda")
    lens = torch.tensor([r.length for r in sample], dtype=torch.int64, device="cuda")
    kidx = torch.tensor([r.key_idx for r in sample], dtype=torch.int32, device="cuda")
    one = hh.to_u64(hh.hash(keys, data, offs, lens, kidx, 4))
    for i, r in enumerate(sample):
        assert tuple(int(x) for x in one[i][:r.width]) == r.result
