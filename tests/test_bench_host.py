"""Host-side logic of bench.py (no GPU): argument checks, the per-kernel
source hashes that gate the reuse of counter summaries, and the shape of the
summaries committed under profiles/."""
import glob
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + list(args),
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_reason():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_prf_path_needs_the_prf_workload():
    r = _run("--path", "prf")
    assert r.returncode == 2
    assert "prf_counters" in r.stderr


def test_every_path_names_a_kernel_with_sources():
    for path, kernel in bench.PATH_KERNEL.items():
        assert kernel in bench.KERNEL_SOURCES, path
        for rel in bench.KERNEL_SOURCES[kernel]:
            assert os.path.exists(os.path.join(ROOT, rel)), rel


def test_source_hash_is_per_kernel_and_stable():
    a = bench.kernel_source_sha("hh_long_kernel")
    assert a == bench.kernel_source_sha("hh_long_kernel")
    assert len(a) == 16 and int(a, 16) >= 0
    # the persistent kernel and the single-launch kernels build from
    # different files, so their hashes differ
    assert a != bench.kernel_source_sha("hh_thread_kernel")
    assert bench.kernel_source_sha("hh_thread_kernel") == bench.kernel_source_sha("hh_prf_kernel")


def test_workload_names_resolve():
    for name in ("lognormal", "plain_fixed", "short_mixed", "prf_counters"):
        assert callable(getattr(__import__("paper_1612_06257_amd.workloads",
                                           fromlist=[name]), name))


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(ROOT, "profiles", "*_valu.json")) +
                                        glob.glob(os.path.join(ROOT, "profiles",
                                                               "*_traffic.json"))))
def test_committed_counter_summaries_are_well_formed(path):
    rec = json.load(open(path))
    base = rec["kernel"].split("::")[-1].split("<")[0]
    assert base in bench.KERNEL_SOURCES
    name = os.path.basename(path)
    assert name.startswith(base + "_")
    assert len(rec["source_sha"]) == 16
    assert rec["workload"]
    if base == "hh_long_kernel":
        # the bucketed kernel's launches depend on the tuning it ran with
        assert set(rec["tuning"]) == set(bench.TUNING_KEYS)
    if name.endswith("_valu.json"):
        c = rec["per_launch"]
        assert c["SQ_INSTS_VALU"] > 0 and c["SQ_WAVES"] > 0
        assert "rocprofv3 --pmc" in rec["command"]
    else:
        assert rec["hbm_bytes_per_launch"] > 0
        assert 0.5 < rec["fetch_scale"] < 4 and 0.5 < rec["write_scale"] < 4


def test_tuning_argument_is_checked():
    assert bench.parse_tuning('{"lane4_min_bytes": 0}') == {"lane4_min_bytes": 0}
    for bad in ('[]', '{}', '{"ring": 72}', '{"long_ring": "72"}', '{"use_graph": true}', 'x'):
        with pytest.raises(ValueError):
            bench.parse_tuning(bad)
    r = _run("--tuning", '{"ring": 72}')
    assert r.returncode == 2 and "unknown fields" in r.stderr


def test_summaries_apply_only_to_launches_like_theirs():
    tuning = {"lane4_min_bytes": 0, "waves_per_cu": 4, "use_graph": 0, "long_ring": 72,
              "isolate_long": 1}
    rec = {"source_sha": bench.kernel_source_sha("hh_long_kernel"), "workload": "w",
           "tuning": dict(tuning)}
    assert bench.profile_applies(rec, "hh_long_kernel", "w", tuning)
    assert not bench.profile_applies(rec, "hh_long_kernel", "other", tuning)
    assert not bench.profile_applies(rec, "hh_long_kernel", "w", dict(tuning, long_ring=96))
    assert not bench.profile_applies(dict(rec, tuning=None), "hh_long_kernel", "w", tuning)
    assert not bench.profile_applies(dict(rec, source_sha="0" * 16), "hh_long_kernel", "w",
                                     tuning)
    assert not bench.profile_applies(None, "hh_long_kernel", "w", tuning)
    # the single-launch kernels do not read the tuning
    rec1 = {"source_sha": bench.kernel_source_sha("hh_thread_kernel"), "workload": "w"}
    assert bench.profile_applies(rec1, "hh_thread_kernel", "w", dict(tuning, long_ring=96))


def test_default_tuning_is_the_library_default():
    from paper_1612_06257_amd import hh
    assert hh.get_tuning() == bench.DEFAULT_TUNING


def test_summary_file_names_carry_non_default_tuning():
    d = dict(bench.DEFAULT_TUNING)
    assert bench.profile_file("hh_long_kernel", "lognormal", "traffic", d).endswith(
        "hh_long_kernel_lognormal_traffic.json")
    assert bench.profile_file("hh_long_kernel", "lognormal", "valu",
                              dict(d, lane4_min_bytes=0)).endswith(
        "hh_long_kernel_lognormal_lane4_min_bytes0_valu.json")
    assert bench.tuning_tag(dict(d, long_ring=96, lane4_min_bytes=0)) == \
        "_lane4_min_bytes0_long_ring96"


def test_binding_roof_names_the_roof_that_binds():
    # the longest chain covering most of the kernel binds it
    assert bench.binding_roof(0.23, 0.12, 1.13, 1.16) == ("critical_path", 1.13 / 1.16)
    # VALU above HBM with a short chain: the integer ALUs bind
    assert bench.binding_roof(0.2, 0.55, 0.001, 0.025) == ("alu", 0.55)
    # HBM above VALU
    assert bench.binding_roof(0.6, 0.4, None, 1.0) == ("hbm", 0.6)
    # nothing near a roof: a launch too small to fill the chip
    assert bench.binding_roof(0.09, 0.02, 0.0015, 0.0055) == ("latency", 0.0015 / 0.0055)
    assert bench.binding_roof(0.12, 0.09, 0.0015, 0.0043) == ("latency", 0.0015 / 0.0043)
    assert bench.binding_roof(None, None, None, None) == ("hbm", None)
