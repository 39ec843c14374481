"""Microbenchmarks behind the roofline figures (needs the GPU).

    python -m paper_1612_06257_amd.microbench [--json out.jsonl]

* chain:   cycles per Update of one wave running a long serial chain of
           Updates on register data, in the four-threads-per-message (quad),
           two-threads-per-message (pair) and one-thread-per-message layouts,
           alone and with other waves sharing the chip, with and without
           s_setprio on the measured waves.
           This is the per-message critical path: a message is one serial
           chain of ceil(L/32)+4 Updates.
* op rate: aggregate rate of each VALU instruction the Update uses, in
           lane-operations per second.
* read:    streaming HBM read bandwidth with 16-byte loads.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
PROBE_LIB = os.path.join(_PKG, "libhh_probe.so")
OPS = ["u64_add", "mad_u64_u32", "perm_b32", "xor_b32", "mov_dpp", "alignbyte_b32"]

_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64


def probe_lib() -> ctypes.CDLL:
    if not os.path.exists(PROBE_LIB):
        raise RuntimeError("libhh_probe.so is not built; run python -m paper_1612_06257_amd.build")
    L = ctypes.CDLL(PROBE_LIB)
    L.hh_probe_chain.argtypes = [ctypes.c_int, _u32, _u32, _u32, _vp, _vp, _vp]
    L.hh_probe_op_rate.argtypes = [ctypes.c_int, _u32, _u32, _vp, _vp]
    L.hh_probe_read.argtypes = [_vp, _u64, _u32, _vp, _vp]
    L.hh_probe_copy.argtypes = [_vp, _vp, _u64, _u32, _vp]
    L.hh_probe_absorb.argtypes = [ctypes.c_int, _vp, _u64, _u64, _u32, _u32, _u32, _vp, _vp, _vp]
    for f in ("hh_probe_chain", "hh_probe_op_rate", "hh_probe_read", "hh_probe_copy",
              "hh_probe_absorb"):
        getattr(L, f).restype = ctypes.c_int
    return L


def _stream():
    return _vp(torch.cuda.current_stream().cuda_stream)


def _time(fn, reps=5):
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


LAYOUTS = {"thread": 0, "quad": 1, "pair": 2}


def chain(L, layout: str, n_updates: int, n_waves: int, prio_waves: int = 0):
    cycles = torch.zeros(n_waves, dtype=torch.int64, device="cuda")
    sink = torch.zeros(64 * n_waves, dtype=torch.int64, device="cuda")

    def go():
        rc = L.hh_probe_chain(LAYOUTS[layout], n_updates, n_waves, prio_waves,
                              _vp(cycles.data_ptr()), _vp(sink.data_ptr()), _stream())
        assert rc == 0, rc

    ms = _time(go, reps=3)
    c = cycles.cpu().numpy().astype(np.float64) / n_updates
    rec = {"kind": "chain", "layout": layout, "n_waves": n_waves,
           "prio_waves": prio_waves, "n_updates": n_updates, "kernel_ms": ms,
           "cycles_per_update_median": float(np.median(c)),
           "cycles_per_update_max": float(c.max()), "cycles_per_update_min": float(c.min())}
    if prio_waves:
        rec["cycles_per_update_prio_max"] = float(c[:prio_waves].max())
        rec["cycles_per_update_rest_median"] = float(np.median(c[prio_waves:]))
    # wall time of the whole launch per Update of the slowest wave (ns)
    rec["ns_per_update_wall"] = ms * 1e6 / n_updates
    return rec


def absorb(L, ring: int, npk: int, n_waves: int, misalign: int, buf=None):
    """Cycles per Update of the production quad packet loop reading memory."""
    msg_bytes = 32 * npk + 64
    need = 16 * n_waves * msg_bytes
    if buf is None or buf.numel() < need:
        buf = torch.empty(need, dtype=torch.uint8, device="cuda")
        buf.fill_(0x5A)
    cycles = torch.zeros(n_waves, dtype=torch.int64, device="cuda")
    sink = torch.zeros(64 * n_waves, dtype=torch.int64, device="cuda")

    def go():
        rc = L.hh_probe_absorb(ring, _vp(buf.data_ptr()), buf.numel(), msg_bytes, misalign, npk,
                               n_waves, _vp(cycles.data_ptr()), _vp(sink.data_ptr()), _stream())
        assert rc == 0, rc

    ms = _time(go, reps=3)
    c = cycles.cpu().numpy().astype(np.float64) / npk
    return {"kind": "absorb", "ring": ring, "npk": npk, "n_waves": n_waves,
            "misalign": misalign, "kernel_ms": ms,
            "cycles_per_update_median": float(np.median(c)),
            "cycles_per_update_max": float(c.max())}, buf


def op_rate(L, op: int, n_blocks: int = 2048, iters: int = 256):
    sink = torch.zeros(256 * n_blocks, dtype=torch.int64, device="cuda")

    def go():
        rc = L.hh_probe_op_rate(op, iters, n_blocks, _vp(sink.data_ptr()), _stream())
        assert rc == 0, rc

    ms = _time(go)
    lane_ops = 256.0 * n_blocks * iters * 16 * 8
    return {"kind": "op_rate", "op": OPS[op], "kernel_ms": ms,
            "lane_ops_per_s": lane_ops / (ms * 1e-3)}


def read_bw(L, gib: float = 4.0, n_blocks: int = 8192):
    nbytes = int(gib * 2**30) // 16 * 16
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(7)
    sink = torch.zeros(256 * n_blocks, dtype=torch.int64, device="cuda")

    def go():
        rc = L.hh_probe_read(_vp(src.data_ptr()), nbytes, n_blocks, _vp(sink.data_ptr()), _stream())
        assert rc == 0, rc

    ms = _time(go)
    return {"kind": "read", "bytes": nbytes, "kernel_ms": ms, "GBps": nbytes / (ms * 1e6)}


def copy(L, nbytes: int, n_blocks: int = 8192, reps: int = 1):
    """Run the plain copy kernel `reps` times (counter calibration)."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(3)
    dst = torch.empty_like(src)
    for _ in range(reps):
        rc = L.hh_probe_copy(_vp(src.data_ptr()), _vp(dst.data_ptr()), nbytes, n_blocks, _stream())
        assert rc == 0, rc
    torch.cuda.synchronize()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--json", default=None)
    ap.add_argument("--summary", default=None, help="write the key figures as JSON here")
    ap.add_argument("--absorb", action="store_true", help="only the packet-loop probe")
    ap.add_argument("--copy-only", type=int, default=0,
                    help="only run the copy kernel on this many bytes (for counters)")
    args = ap.parse_args(argv)
    L = probe_lib()
    if args.copy_only:
        copy(L, args.copy_only, reps=3)
        print("copied %d bytes x3" % args.copy_only, flush=True)
        return
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    recs = []
    if args.absorb:
        buf = None
        for n_waves, npk in ((1, 32768), (4 * cus, 4096)):
            for misalign in (0, 1):
                for ring in (12, 24, 36, 48, 72, 96):
                    r, buf = absorb(L, ring, npk, n_waves, misalign, buf)
                    recs.append(r)
                    print(json.dumps(r), flush=True)
        _write(args, recs, argv)
        return
    n_up = 20000
    for layout in ("quad", "thread", "pair"):
        for n_waves in (1, cus, 4 * cus, 8 * cus, 16 * cus):
            recs.append(chain(L, layout, n_up, n_waves))
            print(json.dumps(recs[-1]), flush=True)
        # priority: the first cus waves raise their priority, 16/CU in total
        recs.append(chain(L, layout, n_up, 16 * cus, prio_waves=cus))
        print(json.dumps(recs[-1]), flush=True)
    buf = None
    for ring in (12, 24, 36, 48, 72, 96):
        r, buf = absorb(L, ring, 32768, 1, 1, buf)
        recs.append(r)
        print(json.dumps(r), flush=True)
    del buf
    for op in range(len(OPS)):
        recs.append(op_rate(L, op))
        print(json.dumps(recs[-1]), flush=True)
    recs.append(read_bw(L))
    print(json.dumps(recs[-1]), flush=True)
    _write(args, recs, argv)


def _write(args, recs, argv) -> None:
    if args.json:
        with open(args.json, "w") as f:
            for r in recs:
                f.write(json.dumps(r) + "\n")
    if args.summary:
        with open(args.summary, "w") as f:
            json.dump(summarize(recs, "python -m paper_1612_06257_amd.microbench " +
                                " ".join(argv if argv is not None else sys.argv[1:])), f,
                      indent=1)
            f.write("\n")


def summarize(recs, command: str) -> dict:
    """Key figures: single-wave Update time per layout, op rates, HBM read."""
    out = {"command": command}
    for r in recs:
        if r["kind"] == "chain" and r["n_waves"] == 1:
            lay = r["layout"]
            out[lay + "_cycles_per_update"] = r["cycles_per_update_median"]
            out[lay + "_ns_per_update"] = r["ns_per_update_wall"]
        if r["kind"] == "chain" and r["prio_waves"]:
            out[r["layout"] + "_prio_cycles_per_update_with_%d_waves" % r["n_waves"]] = \
                r["cycles_per_update_prio_max"]
        if r["kind"] == "op_rate":
            out["op_rate_" + r["op"]] = r["lane_ops_per_s"]
        if r["kind"] == "read":
            out["hbm_read_GBps"] = r["GBps"]
        if r["kind"] == "absorb" and r["n_waves"] == 1 and r["misalign"] == 1:
            ns = r["kernel_ms"] * 1e6 / r["npk"]
            out["quad_loop_ring%d_cycles_per_update" % r["ring"]] = r["cycles_per_update_median"]
            out["quad_loop_ring%d_ns_per_update" % r["ring"]] = ns
    return out


if __name__ == "__main__":
    sys.exit(main())
