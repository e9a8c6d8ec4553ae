"""Host-side checks of bench.py (CPU only): the oracle baseline splits a run into
iterations by time stamps at the oracle's products with A, which assumes two products in
the first iteration and four in every later one (two CGS2 passes, the A-step Gram, the
fresh A W: Algorithm 3 with CGS2 and Pre-CholQR).  A change of that structure must fail
here, not in the benchmark on the GPU."""

import numpy as np

import bench
import workloads as W
from oracle import ecg as ora


def test_oracle_makes_two_then_four_products_per_iteration():
    p = W.config("poisson64")
    A = bench._StampedA(p.A.to_scipy())
    r = ora.flexible_sre_cg2(A, p.b, p.part, p.t, tol=1e-30, kmax=6)
    assert r.it == 5
    assert len(A.stamps) == 1 + 2 + 4 * (r.it - 1)
    assert np.all(np.diff(A.stamps) >= 0)


def test_cpu_baseline_from_a_short_run_and_a_cgs2_probe():
    p = W.config("aniso3d128", scale=8)  # 16^3, t = 32
    widths = [32] * 10 + [16] * 20
    out = bench.cpu_baseline(p, widths, kmax=5, m_probe=(64, 256))
    assert out["kind"] == "oracle" and out["unit"] == "s" and out["cores"] >= 1
    assert out["value"] > 0 and out["measured_sample_s"] > 0
    assert out["per_column_s"] >= 0 and out["per_iteration_const_s"] >= 0
    assert "first 4 iterations" in out["sample"] and "m=256" in out["sample"]
    # the estimate covers all 30 iterations: at least 29 times the constant part
    assert out["value"] >= 29 * out["per_iteration_const_s"]


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys

    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr
