"""bench.py contract checks that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_request_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_work_model_and_effective_peak():
    sys.path.insert(0, ROOT)
    import bench
    N, NS = 128, 64
    mixed = bench.work_model("slater_sample", N, 1527, 253, 0, True)
    fp64 = bench.work_model("slater_sample", N, 1527, 253, 1, False)
    gemm = 2 * N * NS * NS
    # the three contractions of both spins, 6 x (2 N NS^2) flops per walker and sample: B = C A^-1
    # in FP64, M = X B and W = B M on the FP32 matrix cores in mixed precision
    assert mixed["f64"] == 2 * gemm and mixed["f32_mfma"] == 4 * gemm
    assert set(fp64) == {"f64"} and fp64["f64"] > 6 * gemm
    assert fp64["f64"] - 6 * gemm > mixed["f32"]       # three Gaussian images per axis instead of one
    tot1, _, pk = bench.roofline_numbers(mixed, 1, 1e-3)
    tot2, ach, pk2 = bench.roofline_numbers(mixed, 16384, 1e-3)
    assert tot2 == 16384 * tot1 and pk == pk2
    assert bench.PEAK["f64"] < pk < bench.PEAK["f32"]
    # the sweep: the method's count per move (MO row, ratio, acceptance-weighted Sherman-Morrison
    # update in FP64; basis values and Jastrow change in FP32), and the padded work it executes
    sw = bench.work_model("sweep_half", N, 1527, 253, 0, True, acc=0.5)
    assert sw["f64"] == NS * (2 * N * NS + 2 * NS + 0.5 * 4 * NS * NS)
    assert sw["f32"] == NS * (N * (3 * 5 + 2) + 30 * (N - 1))
    ex = bench.executed_model("sweep_half", N, 1527, 253, 0, True, acc=0.5)
    assert ex["f64"] == 2 * NS * N * NS + 4 * NS ** 3 + 16 * NS * NS
    assert sum(ex.values()) > sum(sw.values())


def test_traffic_is_reported_only_for_the_profiled_workload():
    """The committed counter summary applies to one workload: another size, precision, r_s or the
    one-body term changes every kernel's traffic, so the lookup returns None for them."""
    import json
    sys.path.insert(0, ROOT)
    import bench
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    key = bench.traffic_workload_key("h128", "mixed", 16384)
    assert d["workload"] == key
    expect = d["kernels"]["sweep_half"]["bytes_per_launch"] if d["source_hash"] == bench.kernel_source_hash() else None
    assert bench.measured_traffic("sweep_half", key) == expect
    for other in (bench.traffic_workload_key("h128", "fp64", 16384), bench.traffic_workload_key("h256", "mixed", 32768),
                  bench.traffic_workload_key("h128", "mixed", 8192), bench.traffic_workload_key("h128", "mixed", 16384, 2.5),
                  bench.traffic_workload_key("h128", "mixed", 16384, 0.0, 1.28)):
        assert bench.measured_traffic("sweep_half", other) is None


def test_complex_work_model_and_twist_mesh(oracle):
    """The general-twist kernels' counts (complex multiply-add = 8 flops) and the Monkhorst-Pack
    mesh of the twist leg (the oracle's mesh, symmetric about the origin)."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    N, NS = 128, 64
    sw = bench.work_model("csweep", N, 0, 0, 1, False, acc=0.5)
    move = N * 93 + 8 * N * NS + 8 * NS + 30 * (N - 1) + 0.5 * 16 * NS * NS
    assert sw == {"f64": NS * move + (NS * N * 93 + 8 * NS * N * NS + 8 * NS ** 3) / bench.CREFRESH}
    ex = bench.executed_model("csweep", N, 0, 0, 1, False, acc=0.5)
    assert ex["f64"] == sw["f64"] + NS * 0.5 * 8 * NS * NS
    sl = bench.work_model("cslater_sample", N, 0, 0, 1, False)
    assert sl["f64"] > 48 * N * NS * NS
    mesh = bench.monkhorst_pack(4)
    np.testing.assert_allclose(mesh, oracle.monkhorst_pack(4))
    assert mesh.shape == (64, 3) and np.allclose(mesh.sum(0), 0.0)


def test_three_body_work_model_and_arguments():
    """The three-body kernels' counts in the working precision of the Jastrow terms, the term's
    share of a move in the half-sweep, and the F argument of --j3 / --three-body-leg."""
    import argparse
    import pytest
    sys.path.insert(0, ROOT)
    import bench
    N, NS = 128, 64
    for mixed, unit in ((True, "f32"), (False, "f64")):
        g = bench.work_model("j3_grad", N, 0, 0, 1, mixed)
        f = bench.work_model("j3_forces", N, 0, 0, 1, mixed)
        assert g == {unit: N * N * (26 + bench.J3_VGL + 28)} and f == {unit: N * N * (bench.J3_FULL + 150)}
    assert bench.work_model("j3_init", N, 0, 0, 1, True) == {"f64": N * N * 19}
    a = bench.work_model("sweep_half", N, 0, 0, 1, True, acc=0.5)
    b = bench.work_model("sweep_half", N, 0, 0, 1, True, acc=0.5, three_body=True)
    assert b["f64"] == a["f64"] and b["f32"] - a["f32"] == NS * bench.J3_MOVE * N
    ea = bench.executed_model("sweep_half", N, 0, 0, 1, True, acc=0.5)
    eb = bench.executed_model("sweep_half", N, 0, 0, 1, True, acc=0.5, three_body=True)
    assert eb["f32"] - ea["f32"] == NS * bench.J3_MOVE * N
    assert bench._f3("-0.2,0,0.05") == (-0.2, 0.0, 0.05) and bench._f3("none") is None
    with pytest.raises(argparse.ArgumentTypeError):
        bench._f3("1,2")
    assert bench.traffic_workload_key("h128", "mixed", 16, 2.5, None, (-0.2, 0.0, 0.05)) == \
        "h128 mixed, W=16, b1=2.5, F3=-0.2,0,0.05"


def test_optimisation_work_model():
    """The SR statistics kernel's count: the two-body pairs once each, the one-body pairs only with
    the term, the three-body sums always, in the working precision; the 64 moments of the seven parameters in FP64 (two flops each)."""
    sys.path.insert(0, ROOT)
    import bench
    N = 128
    a = bench.work_model("opt_sample", N, 0, 0, 1, True, one_body=True)
    b = bench.work_model("opt_sample", N, 0, 0, 1, False, one_body=False)
    assert a == {"f64": 128, "f32": N * (N - 1) // 2 * 25 + N * N * 25 + N * N * 24}
    assert b == {"f64": N * (N - 1) // 2 * 25 + N * N * 24 + 128}
