"""The oracle still reproduces the vectors it wrote when it was pinned
(guards against unnoticed drift of the oracle's arithmetic)."""
import oracle
from _golden import load_vectors


def test_oracle_reproduces_frozen_vectors():
    vecs = load_vectors()
    assert len(vecs) > 100
    for key, msg, h in vecs:
        assert oracle.hash256(key, msg) == h
        assert oracle.hash64(key, msg) == h[0]
