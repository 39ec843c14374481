"""Turn rocprofv3 CSV output into the short summaries kept under profiles/.

    python -m paper_1612_06257_amd.profiles_summary stats  <kernel_stats.csv> <out.md> <command>
    python -m paper_1612_06257_amd.profiles_summary traffic <fetch.csv> <write.csv> \
        <copy_fetch.csv> <copy_write.csv> <copy_bytes> <workload> <out.json> [options]
    python -m paper_1612_06257_amd.profiles_summary valu <sq.csv> <workload> <out.json> [options]

options:
  --kernel PREFIX      the kernel to summarise (default hh::hh_long_kernel<1)
  --bench-args ARGS    the bench.py arguments of the profiled runs (recorded
                       in the summary's commands)
  --tuning JSON        the hh_tuning the profiled runs were given with
                       bench.py --tuning, recorded so that a benchmark reuses
                       the figures only for launches made with that tuning
  --width N            output words per message of the profiled runs

`traffic` scales the per-dispatch FETCH_SIZE and WRITE_SIZE (KiB) of the
kernel by the factor that makes the same counters read the known size of a
plain copy kernel, and records the hash of the kernel sources so that a
later benchmark only reuses the figure while the kernel is unchanged.
"""
import csv
import json
import sys


def kernel_stats(path, out, command):
    rows = list(csv.DictReader(open(path)))
    lines = ["# rocprofv3 --kernel-trace --stats", "", "Command: `%s`" % command, "",
             "| kernel | calls | avg us | min us | max us | % |", "|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"].replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
        lines.append("| %s | %s | %.1f | %.1f | %.1f | %.2f |" % (
            name, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    open(out, "w").write("\n".join(lines) + "\n")


def _base(kernel: str) -> str:
    """hh::hh_long_kernel<1, 72> -> hh_long_kernel"""
    return kernel.split("::")[-1].split("<")[0]


def _per_kernel(path):
    agg = {}
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"].replace("(anonymous namespace)::", "")
        agg.setdefault(name.split("(")[0].replace("void ", ""), []).append(
            float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in agg.items()}


def _tuning_arg(tuning):
    return "" if tuning is None else " --tuning '%s'" % json.dumps(tuning, sort_keys=True)


def traffic(fetch, write, copy_fetch, copy_write, copy_bytes, workload, out,
            kernel_prefix="hh::hh_long_kernel<1", tuning=None, bench_args=None, width=1):
    sys.path.insert(0, ".")
    import bench
    f = _per_kernel(fetch)
    w = _per_kernel(write)
    kernel = next(k for k in f if k.startswith(kernel_prefix))
    cf = _per_kernel(copy_fetch)["hh::hh_probe_copy_kernel"]
    cw = _per_kernel(copy_write)["hh::hh_probe_copy_kernel"]
    f_factor = copy_bytes / (cf * 1024.0)
    w_factor = copy_bytes / (cw * 1024.0)
    rec = {
        "kernel": kernel, "workload": workload, "source_sha": bench.kernel_source_sha(_base(kernel)),
        "fetch_kib_per_dispatch": f[kernel], "write_kib_per_dispatch": w[kernel],
        "copy_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
        "fetch_scale": f_factor, "write_scale": w_factor,
        "hbm_bytes_per_launch": f[kernel] * 1024.0 * f_factor + w[kernel] * 1024.0 * w_factor,
        "other_kernels_fetch_kib": {k: v for k, v in f.items() if k != kernel},
        "tuning": tuning, "width": width,
        "commands": [
            "rocprofv3 --pmc FETCH_SIZE -d <dir> -o bench --output-format csv -- python -u bench.py "
            + (bench_args or BENCH_ARGS) + _tuning_arg(tuning),
            "rocprofv3 --pmc WRITE_SIZE -d <dir> -o bench --output-format csv -- python -u bench.py "
            + (bench_args or BENCH_ARGS) + _tuning_arg(tuning),
            "rocprofv3 --pmc FETCH_SIZE -d <dir> -o copy --output-format csv -- python -u -m paper_1612_06257_amd.microbench --copy-only %d" % copy_bytes,
            "rocprofv3 --pmc WRITE_SIZE -d <dir> -o copy --output-format csv -- python -u -m paper_1612_06257_amd.microbench --copy-only %d" % copy_bytes,
        ],
    }
    json.dump(rec, open(out, "w"), indent=1)
    open(out, "a").write("\n")
    return rec


VALU_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_BUSY_CYCLES",
                 "SQ_WAVE_CYCLES", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_INSTS_VMEM_RD",
                 "GRBM_GUI_ACTIVE")


BENCH_ARGS = ("--steps 2 --warmup 1 --no-cpu-baseline --no-plain --no-autotune --no-serving "
              "--no-pipelined")


def valu(path, workload, out, kernel_prefix="hh::hh_long_kernel<1", bench_args=BENCH_ARGS,
         tuning=None, width=1):
    """Per-dispatch means of the SQ counters of one kernel (one rocprofv3
    --pmc run of bench.py with VALU_COUNTERS), with the kernel-source hash."""
    sys.path.insert(0, ".")
    import bench
    per = {}
    for r in csv.DictReader(open(path)):
        k = r["Kernel_Name"].split("(")[0].replace("void ", "")
        if k.startswith(kernel_prefix):
            per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
            kernel = k
    rec = {"kernel": kernel, "workload": workload,
           "source_sha": bench.kernel_source_sha(_base(kernel)),
           "per_launch": {c: sum(v) / len(v) for c, v in sorted(per.items())},
           "launches": len(next(iter(per.values()))),
           "tuning": tuning, "width": width,
           "command": "rocprofv3 --pmc " + " ".join(VALU_COUNTERS) + " -d <dir> -o bench "
                      "--output-format csv -- python -u bench.py " + bench_args
                      + _tuning_arg(tuning)}
    json.dump(rec, open(out, "w"), indent=1)
    open(out, "a").write("\n")
    return rec


def _options(argv):
    """Split --kernel/--bench-args/--tuning/--width from the positional
    arguments."""
    opts = {"kernel_prefix": "hh::hh_long_kernel<1", "bench_args": None, "tuning": None,
            "width": 1}
    names = {"--kernel": "kernel_prefix", "--bench-args": "bench_args", "--tuning": "tuning",
             "--width": "width"}
    pos = []
    i = 0
    while i < len(argv):
        if argv[i] in names:
            key = names[argv[i]]
            val = argv[i + 1]
            opts[key] = json.loads(val) if key == "tuning" else int(val) if key == "width" else val
            i += 2
        else:
            pos.append(argv[i])
            i += 1
    return pos, opts


if __name__ == "__main__":
    pos, opts = _options(sys.argv[1:])
    if pos[0] == "stats":
        kernel_stats(pos[1], pos[2], pos[3])
    elif pos[0] == "valu":
        if opts["bench_args"] is None:
            opts["bench_args"] = BENCH_ARGS
        print(json.dumps(valu(pos[1], pos[2], pos[3], **opts), indent=1))
    else:
        print(json.dumps(traffic(pos[1], pos[2], pos[3], pos[4], int(pos[5]), pos[6], pos[7],
                                 **opts), indent=1))
