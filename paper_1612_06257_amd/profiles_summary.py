"""Turn rocprofv3 CSV output into the short summaries kept under profiles/.

    python -m paper_1612_06257_amd.profiles_summary stats  <kernel_stats.csv> <out.md> <command>
    python -m paper_1612_06257_amd.profiles_summary traffic <fetch.csv> <write.csv> \
        <copy_fetch.csv> <copy_write.csv> <copy_bytes> <workload> <out.json>
    python -m paper_1612_06257_amd.profiles_summary valu <sq.csv> <workload> <out.json> \
        [<kernel prefix> [<bench.py arguments of the profiled run>]]

`traffic` and `valu` take `--tuning JSON`: the hh_tuning the profiled runs
were given with `bench.py --tuning`, recorded so that a benchmark reuses the
figures only for launches made with that tuning.

`traffic` scales the per-dispatch FETCH_SIZE and WRITE_SIZE (KiB) of
hh_long_kernel by the factor that makes the same counters read the known size
of a plain copy kernel, and records the hash of the kernel sources so that a
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
        name = r["Name"].split("(")[0].replace("void ", "")
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
        agg.setdefault(r["Kernel_Name"].split("(")[0].replace("void ", ""), []).append(
            float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in agg.items()}


def _tuning_arg(tuning):
    return "" if tuning is None else " --tuning '%s'" % json.dumps(tuning, sort_keys=True)


def traffic(fetch, write, copy_fetch, copy_write, copy_bytes, workload, out,
            kernel_prefix="hh::hh_long_kernel<1", tuning=None):
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
        "tuning": tuning,
        "commands": [
            "rocprofv3 --pmc FETCH_SIZE -d <dir> -o bench --output-format csv -- python -u bench.py "
            + BENCH_ARGS + _tuning_arg(tuning),
            "rocprofv3 --pmc WRITE_SIZE -d <dir> -o bench --output-format csv -- python -u bench.py "
            + BENCH_ARGS + _tuning_arg(tuning),
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
         tuning=None):
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
           "tuning": tuning,
           "command": "rocprofv3 --pmc " + " ".join(VALU_COUNTERS) + " -d <dir> -o bench "
                      "--output-format csv -- python -u bench.py " + bench_args
                      + _tuning_arg(tuning)}
    json.dump(rec, open(out, "w"), indent=1)
    open(out, "a").write("\n")
    return rec


if __name__ == "__main__":
    argv = sys.argv[1:]
    tuning = None
    if "--tuning" in argv:
        i = argv.index("--tuning")
        tuning = json.loads(argv[i + 1])
        del argv[i:i + 2]
    if argv[0] == "stats":
        kernel_stats(argv[1], argv[2], argv[3])
    elif argv[0] == "valu":
        print(json.dumps(valu(*argv[1:6], tuning=tuning), indent=1))
    else:
        print(json.dumps(traffic(argv[1], argv[2], argv[3], argv[4], int(argv[5]), argv[6],
                                 argv[7], tuning=tuning), indent=1))
