"""ecg_solve_noalloc (the solve in the library's static device workspace) against ecg_solve
with a caller workspace, through the C ABI: two calls in a row, the second on a smaller
problem, each compared with ecg_solve on the same inputs (iterations, residual history and
solution bitwise: the same kernels in the same order), plus the size limit."""

import numpy as np
import pytest

import workloads as W
from oracle import ecg as ora

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_2305_19013_amd import ecg

    ecg.lib()
    return torch, torch.device("cuda:0"), ecg


def _pair(env, p, **kw):
    torch, dev, ecg = env
    op = ecg.Operator.from_csr(p.A)
    P = ecg.Partition(p.part, p.t)
    b = torch.from_numpy(p.b).to(dev)
    opts = ecg.options(tol=p.tol, **kw)
    x_ws = torch.zeros_like(b)
    rep_ws, h_ws = ecg.solve(op, P, b, x_ws, opts, rho_hist=True)
    x_na = torch.zeros_like(b)
    rep_na, h_na = ecg.solve_noalloc(op, P, b, x_na, opts, rho_hist=True)
    torch.cuda.synchronize()
    return rep_ws, h_ws, x_ws.cpu().numpy(), rep_na, h_na, x_na.cpu().numpy()


def test_noalloc_matches_workspace_solve_twice_then_limit(env):
    torch, dev, ecg = env
    big = W.config("poisson64")  # 64 x 64, t = 8
    small = W.config("poisson64", scale=2)  # 32 x 32, t = 8
    for p, kw in ((big, dict(kmax=200)), (small, dict(kmax=120, reduce=ora.REDUCE_ONCE, switch_tol=1e-4, t_min=4))):
        print(f"noalloc: {p.name} n={p.n} t={p.t} {kw}", flush=True)
        assert ecg.workspace_size(ecg.Operator.from_csr(p.A), ecg.Partition(p.part, p.t), ecg.options(**kw)) <= 64 << 20
        rep_ws, h_ws, x_ws, rep_na, h_na, x_na = _pair(env, p, **kw)
        assert rep_na["status"] == rep_ws["status"] == "ok"
        for key in ("iters", "switch_iters", "vectors_stored", "deflated_cols", "t_final"):
            assert rep_na[key] == rep_ws[key], key
        assert np.array_equal(h_na, h_ws)
        assert np.array_equal(x_na, x_ws)
        assert rep_na["relres_true"] <= 1.01e-8
        # and both against the oracle at the parity bar
        ref = ora.flexible_sre_cg2(p.A.to_scipy(), p.b, p.part, p.t, tol=p.tol, **kw)
        assert rep_na["iters"] == ref.it
        assert np.linalg.norm(x_na - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    # a solve that needs more than the static 64 MiB is refused before any device work
    p = big
    op = ecg.Operator.from_csr(p.A)
    P = ecg.Partition(p.part, p.t)
    b = torch.from_numpy(p.b).to(dev)
    x = torch.full_like(b, 3.0)
    with pytest.raises(ecg.EcgError) as e:
        ecg.solve_noalloc(op, P, b, x, ecg.options(tol=p.tol, kmax=20000))
    assert e.value.status == ecg.ECG_ENOMEM
    torch.cuda.synchronize()
    assert bool(torch.all(x == 3.0))
