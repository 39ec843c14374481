"""Benchmark: batched HighwayHash-64 on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload lognormal]
                    [--path auto|bucketed|lane1|lane4|prf] [--width 1|2|4]

One step = one hh_hash64 call over the whole batch (planner + every hash: key
setup, packets, remainder, finalization, output), inputs already resident in
HBM.  The default workload is the uneven-length batch: 2^16 messages with
log-normal lengths (median 4 KiB, sigma 2.15, clipped to [1 B, 1 MiB]),
about 2.17 GB packed into one buffer, one key.

Printed as one JSON line:
  value        GB/s hashed, batched path (total message bytes / time per step)
  plain        the same batch through the plain one-thread-per-message kernel,
               one launch per distinct length (the baseline the batched path
               is measured against), plus single-launch variants
  roofline     the dominant kernel (the persistent long-message kernel on the
               batched path, else the path's one kernel): algorithmic bytes
               per launch / its mean duration, timed with HIP events on the
               launch stream (around each persistent launch; around all the
               back-to-back launches of a one-kernel path); valu_roofline the same
               kernel's counted VALU lane-ops over that duration.
               roofline.bound names the roof that binds: "critical_path"
               when the longest message's chain covers at least 0.8 of the
               kernel's time; "latency" when the HBM, VALU and chain
               fractions all stay below 0.5 (a launch too small to fill the
               chip); else "alu" when the VALU fraction exceeds the HBM
               fraction, else "hbm"; bound_frac is that roof's fraction
               (achieved/peak/frac/traffic stay the HBM figures)
  critical_path  the longest message's serial Update chain at the measured
               single-wave Update time
  pipelined    the same steps issued round-robin on 2 and 3 streams (each
               stream its own workspace and output): independent batches
               overlap, the next batch's bulk filling the CUs that one
               batch's few longest chains leave idle; every output is checked
               against the single-stream result
  cpu_baseline the CPU oracle on the host's cores, same batch
  serving      the serving loop on a 10,000-request trace (power-law lengths
               on [8 B, 16 MiB], 64 keys, widths 1/2/4, 32 GiB budget):
               saturation, then Poisson loads at 25/50/80% of the saturation
               request rate, GB/s and p50/p99 request latency; every result
               of every point is checked against the oracle in the CPU
               baseline leg (serving.parity).  --no-serving skips it.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time
from typing import Optional

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GB/s hashed (HighwayHash-64) batched vs plain on 1 MI355X; p99 request latency"
HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, published
OUT_BYTES = 8                   # bytes per output word (HighwayHash-64: one word)
# roofline.bound is "critical_path" when the longest chain covers at least
# this fraction of the dominant kernel's time
CRITICAL_BOUND_FRAC = 0.8
# ... and "latency" when the HBM, VALU and chain fractions all stay below this
LATENCY_BOUND_FRAC = 0.5
KEY_BYTES = 32
PROFILE_DIR = os.path.join(ROOT, "profiles")
# integer VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one lane-op per
# lane per cycle for a full-rate instruction
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
# the paper's own figures (Sec. 5, cycles-per-byte table): HighwayHash AVX2 on
# one core of a Xeon E5-2690 v3 at 2.6 GHz; context only
PAPER_CONTEXT = {"cpu": "Xeon E5-2690 v3, one core, 2.6 GHz, AVX2",
                 "cycles_per_byte": {"8": 7.34, "64": 0.95, "1024": 0.24},
                 "GBps_at_1024_bytes": round(2.6 / 0.24, 2)}
CHAIN_FILE = os.path.join(PROFILE_DIR, "microbench_update_chain.json")
_CSRC = "paper_1612_06257_amd/csrc/"
# the sources each kernel is compiled from: their hash gates the reuse of that
# kernel's counter summaries under profiles/
KERNEL_SOURCES = {
    "hh_long_kernel": [_CSRC + "hh_batched.hip", _CSRC + "hh_msg.hpp", _CSRC + "hh_device.hpp"],
    "hh_thread_kernel": [_CSRC + "hh_kernels.hip", _CSRC + "hh_msg.hpp", _CSRC + "hh_device.hpp"],
    "hh_quad_kernel": [_CSRC + "hh_kernels.hip", _CSRC + "hh_msg.hpp", _CSRC + "hh_device.hpp"],
    "hh_prf_kernel": [_CSRC + "hh_kernels.hip", _CSRC + "hh_msg.hpp", _CSRC + "hh_device.hpp"],
}
# the kernel that does the hashing on each path
PATH_KERNEL = {"auto": "hh_long_kernel", "bucketed": "hh_long_kernel",
               "lane1": "hh_thread_kernel", "lane4": "hh_quad_kernel", "prf": "hh_prf_kernel"}


TUNING_KEYS = ("lane4_min_bytes", "waves_per_cu", "use_graph", "long_ring", "isolate_long")
# the library's defaults (hh_get_tuning before any hh_set_tuning)
DEFAULT_TUNING = {"lane4_min_bytes": 128, "waves_per_cu": 4, "use_graph": 0, "long_ring": 72,
                  "isolate_long": 1}


def parse_tuning(text: str) -> dict:
    """hh_tuning fields from a JSON object; unknown fields or non-integer
    values raise ValueError (the library checks the ranges)."""
    try:
        t = json.loads(text)
    except ValueError as e:
        raise ValueError("not JSON: %s" % e)
    if not isinstance(t, dict) or not t:
        raise ValueError("expected a JSON object of hh_tuning fields")
    bad = sorted(set(t) - set(TUNING_KEYS))
    if bad:
        raise ValueError("unknown fields %s (known: %s)" % (bad, ", ".join(TUNING_KEYS)))
    if not all(isinstance(v, int) and not isinstance(v, bool) for v in t.values()):
        raise ValueError("values must be integers")
    return t


def profile_applies(rec, kernel: str, workload_name: str, tuning: dict, width: int = 1) -> bool:
    """A committed counter summary describes the timed launches only if it
    was taken from the same kernel sources on the same workload with the
    same output width and, for the bucketed path's kernel (the only one the
    tuning changes), with the same tuning."""
    if not rec or rec.get("source_sha") != kernel_source_sha(kernel):
        return False
    if rec.get("workload") != workload_name or rec.get("width", 1) != width:
        return False
    if kernel == "hh_long_kernel":
        return rec.get("tuning") == {k: tuning[k] for k in TUNING_KEYS}
    return True


def tuning_tag(tuning: Optional[dict]) -> str:
    """File-name tag of a tuning: its fields that differ from the library
    defaults, e.g. "_lane4_min_bytes0" (empty for the defaults)."""
    if not tuning:
        return ""
    return "".join("_%s%d" % (k, tuning[k]) for k in TUNING_KEYS
                   if k in tuning and tuning[k] != DEFAULT_TUNING[k])


def width_tag(width: int) -> str:
    """File-name tag of an output width other than one word, e.g. "_w4"."""
    return "" if width == 1 else "_w%d" % width


def profile_file(kernel: str, workload: str, what: str, tuning: Optional[dict] = None,
                 width: int = 1) -> str:
    """Path of a committed counter summary; summaries of the bucketed
    kernel taken with other than the default tuning carry its tag, and
    summaries of wider outputs their width."""
    return os.path.join(PROFILE_DIR, "%s_%s%s%s_%s.json" % (kernel, workload, tuning_tag(tuning),
                                                            width_tag(width), what))


def find_profile(kernel: str, workload: str, what: str, workload_name: str, tuning: dict,
                 width: int = 1):
    """The committed summary that describes launches of `kernel` on this
    workload with this tuning and output width, or None."""
    for t in ((tuning,) if kernel == "hh_long_kernel" else ()) + (None,):
        rec = load_json(profile_file(kernel, workload, what, t, width))
        if profile_applies(rec, kernel, workload_name, tuning, width):
            return rec
    return None


def binding_roof(hbm_frac, valu_frac, critical_ms, kernel_ms):
    """(bound, bound_frac): the roof that binds the dominant kernel.  A chain
    that covers at least CRITICAL_BOUND_FRAC of the kernel's time binds it
    (its fraction: chain floor / kernel time).  When no roof reaches
    LATENCY_BOUND_FRAC the launch is too small to fill the chip and latency
    binds ("latency", with the chain's fraction, the nearest floor).
    Otherwise the larger of the VALU and HBM fractions names the roof."""
    crit = critical_ms / kernel_ms if critical_ms and kernel_ms else None
    if crit is not None and crit >= CRITICAL_BOUND_FRAC:
        return "critical_path", crit
    fracs = [f for f in (hbm_frac, valu_frac, crit) if f is not None]
    if fracs and max(fracs) < LATENCY_BOUND_FRAC:
        return "latency", crit
    if valu_frac is not None and (hbm_frac is None or valu_frac > hbm_frac):
        return "alu", valu_frac
    return "hbm", hbm_frac


def kernel_source_sha(kernel: str = "hh_long_kernel") -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def make_workload(name: str):
    from paper_1612_06257_amd import workloads as W
    if name == "lognormal":
        return W.lognormal()
    if name == "plain_fixed":
        return W.plain_fixed()
    if name == "short_mixed":
        return W.short_mixed()
    if name == "prf_counters":
        return W.prf_counters()
    raise SystemExit("unknown workload " + name)


def to_device(b):
    import torch
    k = torch.from_numpy(b.keys).view(torch.int64).cuda()
    d = torch.from_numpy(b.data).cuda()
    o = torch.from_numpy(b.offsets).view(torch.int64).cuda()
    L = torch.from_numpy(b.lengths).view(torch.int64).cuda()
    ki = None if b.key_idx is None else torch.from_numpy(b.key_idx).view(torch.int32).cuda()
    return k, ki, d, o, L


def time_plain(hh, b, dev):
    """The plain kernel, one launch per distinct length, on one stream."""
    import numpy as np
    import torch
    k, ki, d, o, L = dev
    order = np.argsort(b.lengths, kind="stable")
    lens_sorted = b.lengths[order]
    uniq, starts = np.unique(lens_sorted, return_index=True)
    ends = np.append(starts[1:], lens_sorted.size)
    order_t = torch.from_numpy(order.astype(np.int64)).cuda()
    off_sorted = o[order_t].contiguous()
    ki_sorted = None if ki is None else ki[order_t].contiguous()
    out = torch.empty((b.n, 1), dtype=torch.int64, device="cuda")
    lib = hh.lib()
    stream = hh._stream()
    keys_p = hh._ptr(k)
    groups = []
    for Lg, s, e in zip(uniq.tolist(), starts.tolist(), ends.tolist()):
        groups.append((int(Lg), off_sorted[s:e], None if ki_sorted is None else ki_sorted[s:e],
                       out[s:e]))

    def run():
        for Lg, og, kg, outg in groups:
            st = lib.hh_hash64_uniform(keys_p, k.shape[0], hh._ptr(kg), hh._ptr(d), d.numel(),
                                       hh._ptr(og), Lg, og.numel(), hh._ptr(outg), stream)
            if st != 0:
                raise hh.HHError(st, hh.status_string(st))

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    got = np.empty(b.n, dtype=np.uint64)
    got[order] = hh.to_u64(out)[:, 0]
    return {"value": b.total_bytes / sec / 1e9, "unit": "GB/s", "ms": sec * 1e3,
            "launches": len(groups), "kernel": "hh_thread_kernel (one thread per message)"}, got


def time_single_launch(hh, b, dev, path, width=1):
    import torch
    k, ki, d, o, L = dev
    out = torch.empty((b.n, width), dtype=torch.int64, device="cuda")
    hh.hash(k, d, o, L, ki, width, path, out)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        hh.hash(k, d, o, L, ki, width, path, out)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    return {"value": b.total_bytes / sec / 1e9, "unit": "GB/s", "ms": sec * 1e3}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(b, min_seconds: float = 10.0, max_reps: int = 64, single_bytes: int = 1 << 28,
                 width: int = 1):
    """The oracle's threaded batch driver over the whole batch on min(16,
    cores) threads, repeated until at least min_seconds of wall time (the
    median run is the value), plus one thread on a bounded sample (the
    leading messages, about single_bytes, median of 3 runs)."""
    import numpy as np
    import oracle
    threads = min(16, os.cpu_count() or 1)
    runs = []
    t0 = time.perf_counter()
    while True:
        t = time.perf_counter()
        ref = oracle.batch(b.keys, b.key_idx, b.data, b.offsets, b.lengths, width,
                           n_threads=threads)
        runs.append(time.perf_counter() - t)
        if time.perf_counter() - t0 >= min_seconds or len(runs) >= max_reps:
            break
    med = float(np.median(runs))
    # one thread: the leading messages up to about single_bytes
    lens = b.lengths.astype(np.int64)
    m = int(np.searchsorted(np.cumsum(lens), single_bytes)) + 1
    m = max(1, min(m, b.n))
    sample_bytes = int(lens[:m].sum())
    ki = None if b.key_idx is None else b.key_idx[:m]
    one = []
    for _ in range(3):
        t = time.perf_counter()
        oracle.batch(b.keys, ki, b.data, b.offsets[:m], b.lengths[:m], 1, n_threads=1)
        one.append(time.perf_counter() - t)
    return {"value": b.total_bytes / med / 1e9, "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": "the whole batch (%d messages, %d bytes), %d runs, median"
            % (b.n, b.total_bytes, len(runs)),
            "seconds": float(sum(runs)),
            "single_thread": {"value": sample_bytes / float(np.median(one)) / 1e9,
                              "unit": "GB/s", "sample": "the first %d messages (%d bytes), "
                              "3 runs, median" % (m, sample_bytes)},
            "cpu_model": cpu_model(), "hardware_threads": os.cpu_count()}, ref


def serving_parity(trace, results) -> dict:
    """Part of the CPU-baseline leg: the oracle's hash of every request of the
    serving trace (each at its own width, on the host's cores) against the
    result of that request at every load point."""
    import numpy as np
    import oracle
    threads = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    bad = [0] * len(results)
    for w in (1, 2, 4):
        idx = np.flatnonzero(trace.width_words == w)
        if not idx.size:
            continue
        ref = oracle.batch(trace.keys, trace.key_idx[idx], trace.data, trace.offsets[idx],
                           trace.lengths[idx], w, n_threads=threads)
        for p, res in enumerate(results):
            got = res[idx, :w]
            bad[p] += int(np.count_nonzero(np.any(got != ref, axis=1)))
    return {"parity": "bit-exact" if not any(bad) else "MISMATCH",
            "requests_checked_per_point": int(trace.n), "mismatches_per_point": bad,
            "oracle_seconds": time.perf_counter() - t0, "oracle_threads": threads}


def load_json(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="lognormal",
                    choices=["lognormal", "plain_fixed", "short_mixed", "prf_counters"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving loop run")
    ap.add_argument("--no-pipelined", action="store_true",
                    help="skip the multi-stream run (profiles of the one-stream launches)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the library defaults instead of the autotuned setting")
    ap.add_argument("--tuning", default=None, metavar="JSON",
                    help="time the bucketed path with these hh_tuning fields (the others "
                         "keep the library defaults) instead of the autotuned setting")
    ap.add_argument("--path", default=None, choices=sorted(PATH_KERNEL),
                    help="time this path with the library's tuning instead of the autotuned "
                         "one (prf: the counter-mode kernel, prf_counters workload only)")
    ap.add_argument("--width", type=int, default=1, choices=[1, 2, 4],
                    help="output words per message: 1 (HighwayHash-64, the default), 2 or 4 "
                         "(the plain one-launch-per-length baseline is 64-bit only and is "
                         "skipped for wider outputs)")
    args = ap.parse_args(argv)
    if args.path == "prf" and args.workload != "prf_counters":
        ap.error("--path prf needs --workload prf_counters")
    fixed_tuning = None
    if args.tuning is not None:
        try:
            fixed_tuning = parse_tuning(args.tuning)
        except ValueError as e:
            ap.error("--tuning: %s" % e)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: messages are independent and would shard "
              "across GPUs by bytes, but this build has no multi-GPU path", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_1612_06257_amd import hh

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    hh.lib()
    t_gen = time.perf_counter()
    b = make_workload(args.workload)
    gen_s = time.perf_counter() - t_gen
    dev = to_device(b)
    k, ki, d, o, L = dev
    width = args.width
    out = torch.empty((b.n, width), dtype=torch.int64, device="cuda")

    print("[bench] workload %s: %d messages, %d bytes (generated in %.1f s)"
          % (b.name, b.n, b.total_bytes, gen_s), file=sys.stderr, flush=True)
    # the timed steps run on a private stream (hipGraph capture needs one)
    stream = torch.cuda.Stream()
    tuned = None
    path = args.path or "auto"
    if fixed_tuning is not None:
        hh.set_tuning(**dict(hh.get_tuning(), **fixed_tuning))
        tuned = {"fixed": fixed_tuning}
    elif not args.no_autotune and args.path is None:
        from paper_1612_06257_amd import autotune
        tuned = autotune.tune(k, d, o, L, ki, width, cache_path=None)
        path = tuned["path"]
        if path == "bucketed":
            hh.set_tuning(**dict(hh.get_tuning(), **{x: tuned[x] for x in autotune.TUNING_KEYS}))
        print("[bench] autotuned: %s" % json.dumps(tuned), file=sys.stderr, flush=True)
    kernel = PATH_KERNEL[path]

    # the steps make the C call with arguments checked and marshalled once
    # (as a C caller would); the PRF takes no per-message arguments
    call = None if path == "prf" else hh.prepare(k, d, o, L, ki, width, path, out, stream)

    def step():
        if call is None:
            hh.prf(k, b.n, 0, width, out)
        else:
            call()

    # no cyclic-collector pass inside the timed launches (a full pass stops
    # the host for tens of milliseconds and the GPU would run dry)
    gc.disable()
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step()
        stream.synchronize()
        if kernel == "hh_long_kernel":
            # per-launch HIP events around the persistent kernel; they force
            # direct launches, so the roofline timing is a separate pass
            hh.timing_enable(True)
            hh.timing_collect()
            for _ in range(args.steps):
                step()
            stream.synchronize()
            launches, kernel_ms = hh.timing_collect()
            hh.timing_enable(False)
        else:
            # one kernel per call: one event pair on this stream around the
            # back-to-back launches (an event pair per launch adds its own
            # markers to every launch's time)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                step()
            e1.record()
            stream.synchronize()
            launches, kernel_ms = args.steps, e0.elapsed_time(e1)
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        stream.synchronize()
        sec = time.perf_counter() - t0
    gc.enable()
    ms_per_step = sec * 1e3 / args.steps
    value = b.total_bytes * args.steps / sec / 1e9
    gpu_hash = hh.to_u64(out).copy()
    print("[bench] batched: %.3f ms/step, %.1f GB/s" % (ms_per_step, value), file=sys.stderr,
          flush=True)

    # roofline of the dominant kernel: algorithmic bytes it moves per launch
    # (message bytes read once, 8 bytes per output word, 32 per key) over
    # its mean launch time; the PRF reads no message bytes (its counters are
    # built in registers)
    lengths = b.lengths.astype(np.int64)
    n_keys = int(b.keys.shape[0])
    if kernel == "hh_long_kernel":
        thr = hh.get_tuning()["lane4_min_bytes"]
        mask = lengths >= thr
    else:
        mask = np.ones(lengths.shape, bool)
    msg_bytes = 0 if kernel == "hh_prf_kernel" else int(lengths[mask].sum())
    kernel_bytes = msg_bytes + OUT_BYTES * width * int(mask.sum()) + KEY_BYTES * n_keys
    kernel_ms_mean = kernel_ms / launches if launches else None
    achieved = kernel_bytes / (kernel_ms_mean * 1e6) if kernel_ms_mean else None
    timed_tuning = hh.get_tuning()
    traffic = None
    tr = find_profile(kernel, args.workload, "traffic", b.name, timed_tuning, width)
    if tr:
        traffic = tr.get("hbm_bytes_per_launch")
    roofline = {"bound": "hbm", "kernel": kernel, "achieved": achieved,
                "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBPS) if achieved else None, "traffic": traffic,
                "algorithmic_bytes_per_launch": kernel_bytes,
                "kernel_ms_mean": kernel_ms_mean, "launches_timed": launches}
    # integer-VALU roof of the same kernel, from its counted VALU instructions
    # (each a wave of 64 lane-ops) over the mean launch time measured above
    valu_roof = None
    vc = find_profile(kernel, args.workload, "valu", b.name, timed_tuning, width)
    if vc and kernel_ms_mean:
        c = vc["per_launch"]
        lane_ops = c["SQ_INSTS_VALU"] * 64.0
        valu_roof = {"bound": "alu", "kernel": kernel,
                     "achieved": lane_ops / (kernel_ms_mean * 1e-3) / 1e12,
                     "peak": VALU_PEAK_LANE_OPS / 1e12, "unit": "T lane-ops/s",
                     "frac": lane_ops / (kernel_ms_mean * 1e-3) / VALU_PEAK_LANE_OPS,
                     "valu_insts_per_launch": c["SQ_INSTS_VALU"],
                     "lds_insts_per_launch": c.get("SQ_INSTS_LDS"),
                     "lds_bank_conflict_cycles_per_launch": c.get("SQ_LDS_BANK_CONFLICT")}

    # independent batches on several streams: overlap without changing any
    # batch's work (bucketed path only; the single-launch kernels fill the
    # GPU on their own)
    pipelined = None
    if kernel == "hh_long_kernel" and not args.no_pipelined:
        pipelined = []
        for n_streams in (2, 3):
            # streams measured to run concurrently (the runtime shares a few
            # hardware queues among streams; two on one queue serialise)
            streams = hh.independent_streams(n_streams, avoid=[])
            outs = [torch.empty((b.n, width), dtype=torch.int64, device="cuda")
                    for _ in range(n_streams)]
            for s_, o_ in zip(streams, outs):      # each stream's workspace, warm
                with torch.cuda.stream(s_):
                    hh.hash(k, d, o, L, ki, width, path, o_)
            torch.cuda.synchronize()
            gc.disable()
            t0 = time.perf_counter()
            for i in range(args.steps):
                with torch.cuda.stream(streams[i % n_streams]):
                    hh.hash(k, d, o, L, ki, width, path, outs[i % n_streams])
            torch.cuda.synchronize()
            psec = time.perf_counter() - t0
            gc.enable()
            exact = all(np.array_equal(hh.to_u64(x), gpu_hash) for x in outs)
            pipelined.append({"streams": n_streams, "value": b.total_bytes * args.steps / psec / 1e9,
                              "unit": "GB/s", "ms_per_batch": psec * 1e3 / args.steps,
                              "bit_exact": bool(exact)})
            print("[bench] pipelined on %d streams: %.3f ms/batch, %.1f GB/s" % (
                n_streams, psec * 1e3 / args.steps, b.total_bytes * args.steps / psec / 1e9),
                file=sys.stderr, flush=True)

    # critical path: longest message x measured single-wave Update time
    # (one thread per message on the lane1 and prf paths and for messages
    # below the bucketed path's quad threshold, else four)
    chain = load_json(CHAIN_FILE) or {}
    ring = hh.get_tuning()["long_ring"]
    longest = int(lengths.max()) if lengths.size else 0
    thread_layout = (path in ("lane1", "prf") or
                     (path in ("auto", "bucketed") and longest < hh.get_tuning()["lane4_min_bytes"]))
    if thread_layout:
        t_upd_ns = chain.get("thread_ns_per_update")
    else:
        # the single-launch quad kernel runs a 12-packet ring, the persistent
        # kernel the tuned one
        ring_used = 12 if path == "lane4" else ring
        t_upd_ns = (chain.get("quad_loop_ring%d_ns_per_update" % ring_used)
                    or chain.get("quad_ns_per_update"))
    n_upd = (longest + 31) // 32 + 4
    critical = None
    if t_upd_ns:
        floor_ms = n_upd * t_upd_ns * 1e-6
        critical = {"longest_message_bytes": longest, "updates": n_upd,
                    "layout": "thread" if thread_layout else "quad",
                    "ns_per_update": t_upd_ns, "floor_ms": floor_ms,
                    "frac_of_step": floor_ms / ms_per_step,
                    "frac_of_kernel": floor_ms / kernel_ms_mean if kernel_ms_mean else None}
    bound, bound_frac = binding_roof(roofline["frac"], valu_roof["frac"] if valu_roof else None,
                                     critical["floor_ms"] if critical else None, kernel_ms_mean)
    roofline["bound"] = bound
    roofline["bound_frac"] = bound_frac

    result = {
        "metric": METRIC, "value": value, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": b.name, "n_msgs": b.n, "bytes": b.total_bytes, "seed": b.seed,
                   "output_bits": 64 * width, "path": path, "tuning": hh.get_tuning()},
        "autotune": tuned,
        "messages_per_s": b.n * args.steps / sec,
        "roofline": roofline,
        "valu_roofline": valu_roof,
        "critical_path": critical,
        "pipelined": pipelined,
        "paper_context": PAPER_CONTEXT,
    }

    # the serving run goes first: the 27,560 launches of the plain baseline
    # leave the runtime slower for a while, which the serving latencies see
    result["serving"] = None
    serving_check = None
    if not args.no_serving:
        from paper_1612_06257_amd import serve
        try:
            summary, trace, results = serve.bench_summary()
        except RuntimeError as e:  # a stalled loop: report it, keep the rest of the line
            result["serving"] = {"error": str(e)}
            print("[bench] serving failed: %s" % e, file=sys.stderr, flush=True)
        else:
            result["serving"] = summary
            serving_check = (trace, results)
            pts = [summary["saturation"]] + summary["loads"]
            print("[bench] serving: %s" % json.dumps(
                [{"load": v["load"], "GBps": round(v["GBps"], 1), "p50_ms": round(v["p50_ms"], 3),
                  "p99_ms": round(v["p99_ms"], 2)} for v in pts]), file=sys.stderr, flush=True)

    if not args.no_plain and width == 1:
        plain, plain_hash = time_plain(hh, b, dev)
        plain["bit_exact_with_batched"] = bool(np.array_equal(plain_hash, gpu_hash[:, 0]))
        result["plain"] = plain
        result["batched_over_plain"] = value / plain["value"]
        print("[bench] plain: %d launches, %.1f ms" % (plain["launches"], plain["ms"]),
              file=sys.stderr, flush=True)
    if not args.no_plain:
        result["single_launch"] = {p: time_single_launch(hh, b, dev, p, width)
                                   for p in ("lane1", "lane4")}

    if not args.no_cpu_baseline:
        cb, ref = cpu_baseline(b, width=width)
        result["cpu_baseline"] = cb
        result["parity"] = "bit-exact" if np.array_equal(ref, gpu_hash) else "MISMATCH"
        if serving_check is not None:
            result["serving"].update(serving_parity(*serving_check))
            print("[bench] serving parity: %s" % result["serving"]["parity"], file=sys.stderr,
                  flush=True)
    else:
        result["cpu_baseline"] = None

    print(json.dumps(result))
    ok = (result.get("parity", "bit-exact") == "bit-exact"
          and (result["serving"] or {}).get("parity", "bit-exact") == "bit-exact"
          and "error" not in (result["serving"] or {}))
    return 0 if ok else 3


if __name__ == "__main__":
    sys.exit(main())
