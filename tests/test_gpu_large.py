"""Messages past 4 GiB (GPU required): one message longer than 2^32 bytes,
messages that straddle byte 2^32 of the buffer and messages that start beyond
it, bit-exact with the oracle.  Inside one absorb call the kernels form packet
offsets in 32-bit arithmetic, so a message this long is absorbed in several
calls.  The quad layout runs through the single-launch and bucketed paths and
the streaming-state API; the one-thread layout through the plain kernel, whose
deep ring takes the 2^27 packets in about 20 s (the general one-thread kernel
keeps one packet in flight and would need about a minute)."""
import numpy as np
import pytest
import torch

from _gpu import announce, assert_same, batch_to_device, oracle_ref, require_gpu

pytestmark = pytest.mark.gpu

BIG = (1 << 32) + (1 << 20) + 77  # 2^27 + 32,770 whole packets, remainder 13
START = 3                          # unaligned start of the long message


@pytest.fixture(scope="module")
def hh():
    return require_gpu()


@pytest.fixture(scope="module")
def batch():
    """The long message, messages around byte 2^32 inside it, and short
    messages packed after it (offsets above 2^32); random bytes throughout,
    so a packet read 4 GiB too early would change the hash."""
    rng = np.random.default_rng(1612_0625_7)
    small = rng.integers(0, 5000, 40).astype(np.uint64)
    tail_start = START + BIG
    total = tail_start + int(small.sum()) + 64
    words = np.empty((total + 7) // 8, np.uint64)
    step = 1 << 25
    for w0 in range(0, words.size, step):
        c = min(step, words.size - w0)
        words[w0:w0 + c] = rng.integers(0, 2**64, size=c, dtype=np.uint64)
    data = words.view(np.uint8)[:total]
    two32 = 1 << 32
    offsets = [START, two32 - 1000, two32 - 5, two32, two32 - 64, 0]
    lengths = [BIG, 3001, 5, 32, 64 + 4096 + 9, 0]
    pos = tail_start
    for L in small:
        offsets.append(pos)
        lengths.append(int(L))
        pos += int(L)
    offsets = np.array(offsets, np.uint64)
    lengths = np.array(lengths, np.uint64)
    assert int((offsets + lengths).max()) <= total
    keys = rng.integers(0, 2**64, size=(5, 4), dtype=np.uint64)
    key_idx = rng.integers(0, 5, offsets.size, dtype=np.uint32)
    announce("large: oracle over", total, "bytes")
    want = oracle_ref(4, keys, key_idx, data, offsets, lengths)
    dev = batch_to_device(keys, key_idx, data, offsets, lengths)
    return keys, key_idx, data, offsets, lengths, want, dev


@pytest.mark.parametrize("path", ["lane4", "bucketed"])
def test_long_message_and_offsets_past_4gib(hh, batch, path):
    keys, key_idx, data, offsets, lengths, want, (k, ki, d, o, L) = batch
    announce("large", path)
    got = hh.to_u64(hh.hash(k, d, o, L, ki, width=4, path=path))
    torch.cuda.synchronize()
    assert_same(got, want, "large %s" % path)


def test_plain_kernel_on_the_long_message(hh, batch):
    keys, key_idx, data, offsets, lengths, want, (k, ki, d, o, L) = batch
    announce("large", "uniform")
    out = hh.hash64_uniform(k, d, o[:1], BIG, ki[:1])
    torch.cuda.synchronize()
    assert_same(hh.to_u64(out), want[:1, :1], "large uniform")


def test_state_api_on_the_long_message(hh, batch):
    """Whole packets in one update call (more than 2^27 of them), then the
    remainder and finalization."""
    keys, key_idx, data, offsets, lengths, want, (k, ki, d, o, L) = batch
    announce("large", "state")
    states = hh.state_init(k, 1, ki[:1])
    full = (BIG // 32) * 32
    i64 = dict(dtype=torch.int64, device="cuda")
    hh.state_update(states, d, torch.tensor([START], **i64), torch.tensor([full], **i64))
    out = torch.zeros((1, 4), **i64)
    hh.state_final(states, d, torch.tensor([START + full], **i64),
                   torch.tensor([BIG - full], **i64),
                   torch.tensor([4], dtype=torch.uint8, device="cuda"), out.view(-1))
    torch.cuda.synchronize()
    assert_same(hh.to_u64(out), want[:1, :4], "large state")
