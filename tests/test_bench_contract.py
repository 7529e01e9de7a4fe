"""Host-side checks of the benchmark contract (no device needed): the
one-GPU refusal, the roofline arithmetic on a synthetic statistics record,
and the consistency of the committed profiler records with each other."""
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def _stats(kernels):
    return {"kernels": {n: {"ms": ms, "launches": la, "flops": fl, "bytes": by} for n, (ms, la, fl, by) in kernels.items()}}


def test_roofline_picks_the_largest_single_kernel_and_prices_it():
    st = _stats({"group:sketch_orth": (9000.0, 10, 0.0, 0.0), "k_schur": (2000.0, 100, 4.0e14, 1.0e12),
                 "k_gram": (500.0, 10, 1.0e12, 0.0)})
    rf = bench.roofline_of(st, mixed=True)
    assert rf["kernel"] == "k_schur" and rf["bound"] == "mfma" and rf["unit"] == "TFLOP/s"
    ach = 4.0e14 / 100 / (2000.0 / 1e3 / 100)  # flops per launch / seconds per launch
    assert rf["achieved"] == pytest.approx(ach / 1e12)
    assert rf["frac"] == pytest.approx(ach / bench.FP32_MFMA_PEAK)
    assert rf["avg_launch_ms"] == pytest.approx(20.0)
    assert rf["algorithmic_bytes_per_launch"] == pytest.approx(1.0e10)
    # the FP64 form prices the same kernel against the FP64 matrix-core peak
    rf64 = bench.roofline_of(st, mixed=False)
    assert rf64["bound"] == "mfma" and rf64["frac"] == pytest.approx(ach / bench.FP64_MFMA_PEAK)
    # the mixed form's far products as their own kernel: FP32 matrix cores,
    # and k_schur then holds FP64 products only
    st2 = _stats({"k_schur": (2000.0, 100, 4.0e14, 1.0e12), "k_schur_far": (1000.0, 100, 3.0e14, 0.0)})
    st2["aux"] = {"schur_far_flops": 3.0e14}
    far = bench.price("k_schur_far", st2["kernels"]["k_schur_far"], True, bench._f32_flops(st2, "k_schur_far"))
    assert far["peak"] == pytest.approx(bench.FP32_MFMA_PEAK / 1e12)
    near = bench.price("k_schur", st2["kernels"]["k_schur"], True, bench._f32_flops(st2, "k_schur"))
    assert near["peak"] == pytest.approx(bench.FP64_MFMA_PEAK / 1e12)
    # a memory-bound kernel is priced in bytes against HBM
    rfh = bench.roofline_of(_stats({"k_solve_fwd_upd": (10.0, 10, 0.0, 8.0e10)}), mixed=True)
    assert rfh["bound"] == "hbm" and rfh["frac"] == pytest.approx(8.0e9 / 1e-3 / bench.HBM_PEAK)


def test_committed_profiler_records_agree_with_each_other():
    import glob
    prof = os.path.join(ROOT, "profiles")
    with open(os.path.join(prof, "ifmm_factor_solve_ellipsoid_1M_mixed_kernel_stats.txt")) as fh:
        text = fh.read()
    recs = sorted(glob.glob(os.path.join(prof, "*_hbm_traffic_*.json")))
    assert {os.path.basename(p).split("_hbm")[0] for p in recs} >= {"k_schur", "k_solve_bwd", "k_solve_fwd_upd"}
    for path in recs:
        with open(path) as fh:
            rec = json.load(fh)
        cal = rec["copy_calibration"]
        # the calibration factors are the copy's known bytes over what each counter read
        assert cal["fetch_factor"] == pytest.approx(cal["bytes"] / (cal["fetch_size_kib"] * 1024))
        assert cal["write_factor"] == pytest.approx(cal["bytes"] / (cal["write_size_kib"] * 1024))
        scaled = (rec["fetch_size_kib_per_launch"] * 1024 * cal["fetch_factor"] +
                  rec["write_size_kib_per_launch"] * 1024 * cal["write_factor"])
        assert rec["traffic_bytes_per_launch"] == pytest.approx(scaled)
        assert rec["traffic_over_algorithmic"] == pytest.approx(scaled / rec["algorithmic_bytes_per_launch"])
        # every command the record names runs committed files only
        cmds = list(rec["commands"]) + ([rec["matrix_core_busy"]["command"]] if "matrix_core_busy" in rec else [])
        for cmd in cmds:
            assert "_work" not in cmd and "/root/reference" not in cmd
            for path2 in re.findall(r"(\S+\.py)", cmd):
                assert os.path.exists(os.path.join(ROOT, path2)), path2
        # the kernel statistics were taken on the same kernel sources
        assert rec["kernel_sources_sha256_16"] in text
    m = re.search(r"k_schur<[^>]*>\s+(\d+)\s+([\d.]+) ms\s+avg\s+([\d.]+) us", text)
    with open(os.path.join(prof, "k_schur_hbm_traffic_ellipsoid_1M_mixed.json")) as fh:
        rec = json.load(fh)
    assert m and int(m.group(1)) == rec["launches"]
    bench_avg = float(re.search(r"launches, avg ([\d.]+) ms", text).group(1))
    assert float(m.group(3)) / 1e3 == pytest.approx(bench_avg, rel=0.01)  # trace and in-library timing agree


def test_traffic_lookup_is_keyed_by_form_and_sources():
    assert bench.measured_traffic("k_schur", "no-such-form") is None
    assert bench.measured_traffic("no_such_kernel", "mixed") is None
