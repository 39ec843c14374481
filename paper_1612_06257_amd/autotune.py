"""Autotuner for the batch path.

For a batch (device tensors as for ``hh.hash``) it times candidate settings of
the bucketed path -- split threshold (which messages get four threads each),
persistent residency (waves per CU), prefetch ring depth, hipGraph replay --
and the two single-launch kernels, and keeps the fastest unless the library
defaults are within a small margin of it (the minimum of many noisy timings
beats any fixed setting by about that much on its own).  Results are cached
in a JSON file keyed by device architecture, CU count, output width and a
signature of the batch (message count and the log2 buckets of the mean and
maximum length), so a later batch of the same shape reuses them.

    from paper_1612_06257_amd import autotune
    best = autotune.tune(keys, data, offsets, lengths)      # times candidates
    out = autotune.hash(keys, data, offsets, lengths)       # uses the cache
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time
from typing import Optional

import torch

from . import hh

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "hh_autotune.json")

RINGS = (48, 72, 96)
WAVES_PER_CU = (4, 8)
THRESHOLDS = (0, 64, 128, 512)
GRAPH = (0, 1)
ISOLATE = (1, 0)
TUNING_KEYS = ("long_ring", "waves_per_cu", "lane4_min_bytes", "use_graph", "isolate_long")


def _log2_bucket(x: float) -> int:
    return int(math.floor(math.log2(max(x, 1.0))))


def signature(lengths: torch.Tensor, width: int = 1) -> str:
    props = torch.cuda.get_device_properties(lengths.device)
    n = lengths.numel()
    mean = float(lengths.double().mean()) if n else 0.0
    mx = int(lengths.max()) if n else 0
    arch = getattr(props, "gcnArchName", "unknown").split(":")[0]
    return "%s/cu%d/w%d/n%d/mean%d/max%d" % (arch, props.multi_processor_count, width,
                                             _log2_bucket(n), _log2_bucket(mean),
                                             _log2_bucket(mx))


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path: str, cache: dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time(fn, reps: int) -> float:
    stream = torch.cuda.current_stream()
    fn()
    stream.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    stream.synchronize()
    return (time.perf_counter() - t0) / reps


def candidates():
    for ring, wpc, thr, g, iso in itertools.product(RINGS, WAVES_PER_CU, THRESHOLDS, GRAPH,
                                                    ISOLATE):
        if iso and wpc > 4:
            continue  # isolation needs one workgroup per CU
        yield {"path": "bucketed", "long_ring": ring, "waves_per_cu": wpc,
               "lane4_min_bytes": thr, "use_graph": g, "isolate_long": iso}
    yield {"path": "lane1"}
    yield {"path": "lane4"}


# a candidate replaces the defaults only if it is faster by more than this
# fraction: run-to-run spread of one batch's time is about 1%
DEFAULT_MARGIN = 0.02


def pick(results, defaults: dict, margin: float = DEFAULT_MARGIN):
    """(seconds, candidate) of the choice among the timed (seconds, candidate)
    pairs: the fastest, unless the bucketed path with the `defaults` tuning is
    within `margin` of it; also returns the defaults' time (None if they were
    not timed)."""
    if not results:
        raise ValueError("no timed candidates")
    best = min(results, key=lambda r: r[0])
    default = next((r for r in results if r[1]["path"] == "bucketed" and all(
        r[1][k] == defaults[k] for k in TUNING_KEYS)), None)
    if default is not None and best[0] >= default[0] * (1.0 - margin):
        best = default
    return best[0], best[1], None if default is None else default[0]


def tune(keys, data, offsets, lengths, key_idx=None, width: int = 1, reps: int = 5,
         cache_path: Optional[str] = DEFAULT_CACHE, verbose: bool = False,
         margin: float = DEFAULT_MARGIN) -> dict:
    """Time every candidate on this batch (on a private stream, so that
    hipGraph capture is possible) and cache the choice of `pick`; returns it."""
    saved = hh.get_tuning()
    out = torch.empty((offsets.numel(), width), dtype=torch.int64, device=offsets.device)
    results = []
    stream = torch.cuda.Stream()
    try:
        with torch.cuda.stream(stream):
            for c in candidates():
                if c["path"] == "bucketed":
                    hh.set_tuning(**dict(saved, **{k: v for k, v in c.items() if k != "path"}))
                sec = _time(lambda: hh.hash(keys, data, offsets, lengths, key_idx, width,
                                            c["path"], out), reps)
                results.append((sec, c))
                if verbose:
                    print("autotune %.4f ms %s" % (sec * 1e3, c), flush=True)
    finally:
        hh.set_tuning(**saved)
    sec, best, default = pick(results, saved, margin)
    fastest = min(r[0] for r in results)
    entry = dict(best, ms=sec * 1e3, default_ms=None if default is None else default * 1e3,
                 fastest_ms=fastest * 1e3, margin=margin, candidates=len(results))
    if cache_path:
        cache = _load(cache_path)
        cache[signature(lengths, width)] = entry
        _save(cache_path, cache)
    return entry


def lookup(lengths, width: int = 1, cache_path: str = DEFAULT_CACHE) -> Optional[dict]:
    return _load(cache_path).get(signature(lengths, width))


def hash(keys, data, offsets, lengths, key_idx=None, width: int = 1, out=None,
         cache_path: str = DEFAULT_CACHE):
    """hh.hash with the cached best setting for this batch's signature (the
    library defaults when there is none).  The tuning is process-wide and is
    left set to the cached values."""
    entry = lookup(lengths, width, cache_path)
    if entry is None:
        return hh.hash(keys, data, offsets, lengths, key_idx, width, "auto", out)
    if entry["path"] == "bucketed":
        hh.set_tuning(**dict(hh.get_tuning(), **{k: entry[k] for k in TUNING_KEYS
                                                 if k in entry}))
    return hh.hash(keys, data, offsets, lengths, key_idx, width, entry["path"], out)
