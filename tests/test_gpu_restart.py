"""GPU parity of the restarted variants (Section 3: restart every j iterations, restart on
restartTol, and the restarted flexible variant that empties Q at the halving) against the
FP64 oracle, for SRE-CG2 and MSDO-CG.

Same bar as the other parity tests: iteration counts, restart and switch iterations, the
largest cycle memory exactly; residual histories to 1e-10 rho_0, iterates to 1e-10.
"""

import numpy as np
import pytest

import workloads as W
from oracle import ecg as ora

pytestmark = pytest.mark.gpu

MSDO = 1


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_2305_19013_amd import ecg

    ecg.lib()
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def poisson():
    p = W.config("poisson64")
    return p, p.A.to_scipy()


def _solve(torch, dev, p, **kw):
    from paper_2305_19013_amd import ecg

    op = ecg.Operator.from_csr(p.A)
    P = ecg.Partition(p.part, p.t)
    bt = torch.from_numpy(np.ascontiguousarray(p.b)).to(dev)
    xt = torch.zeros_like(bt)
    rep, rh = ecg.solve(op, P, bt, xt, ecg.options(**kw), rho_hist=True)
    torch.cuda.synchronize()
    return rep, xt.cpu().numpy(), rh


def _same(rep, x, rh, ref):
    assert rep["iters"] == ref.it, (rep["iters"], ref.it)
    assert rep["n_restart"] == len(ref.restart_iters)
    assert rep["restart_iters"] == ref.restart_iters[:8]
    assert rep["switch_iters"] == ref.switch_iters
    assert rep["vectors_stored"] == ref.mem and rep["vectors_peak"] == ref.mem_cycle
    assert np.abs(rh - np.array(ref.rho)).max() <= 1e-10 * ref.rho[0]
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    emax = np.abs(x - ref.x).max() / np.abs(ref.x).max()  # largest entry error
    assert err <= 1e-10 and emax <= 1e-10, (err, emax)


@pytest.mark.parametrize("variant", [0, MSDO])
def test_restart_every_j_parity(torch_dev, poisson, variant):
    torch, dev = torch_dev
    p, A = poisson
    kw = dict(restart=ora.RESTART_EVERY, restart_every=20, kmax=120)
    fn = ora.flexible_msdo_cg if variant == MSDO else ora.flexible_sre_cg2
    ref = fn(A, p.b, p.part, p.t, tol=p.tol, **kw)
    assert ref.restart_iters[:3] == [21, 41, 61] and ref.mem_cycle == 20 * p.t
    rep, x, rh = _solve(torch, dev, p, tol=p.tol, variant=variant, **kw)
    _same(rep, x, rh, ref)


@pytest.mark.parametrize("variant,rtol", [(0, 1e-3), (0, 1e-5), (MSDO, 1e-3)])
def test_restart_tol_parity(torch_dev, poisson, variant, rtol):
    torch, dev = torch_dev
    p, A = poisson
    kw = dict(restart=ora.RESTART_TOL, restart_tol=rtol)
    fn = ora.flexible_msdo_cg if variant == MSDO else ora.flexible_sre_cg2
    ref = fn(A, p.b, p.part, p.t, tol=p.tol, **kw)
    assert len(ref.restart_iters) >= 1 and ref.status == "converged"
    rep, x, rh = _solve(torch, dev, p, tol=p.tol, variant=variant, **kw)
    assert rep["status"] == "ok"
    _same(rep, x, rh, ref)


def test_single_restart_and_restarted_flexible_parity(torch_dev, poisson):
    """The two restarted variants of the memory tables: one restart at restartTol with the
    same t, and the flexible run that also empties Q when it halves."""
    torch, dev = torch_dev
    p, A = poisson
    once = dict(restart=ora.RESTART_TOL, restart_tol=1e-4, max_restarts=1)
    ref = ora.flexible_sre_cg2(A, p.b, p.part, p.t, tol=p.tol, **once)
    rep, x, rh = _solve(torch, dev, p, tol=p.tol, **once)
    _same(rep, x, rh, ref)
    sit = ref.restart_iters[0] - 1
    assert rep["vectors_peak"] == p.t * max(sit, ref.it - sit)
    flex = dict(reduce=ora.REDUCE_ONCE, switch_tol=1e-4, restart_at_switch=True)
    ref = ora.flexible_sre_cg2(A, p.b, p.part, p.t, tol=p.tol, **flex)
    rep, x, rh = _solve(torch, dev, p, tol=p.tol, **flex)
    _same(rep, x, rh, ref)
    assert rep["vectors_peak"] == max(p.t * sit, p.t // 2 * (ref.it - sit))


def test_restart_options_rejected(torch_dev, poisson):
    torch, dev = torch_dev
    p, _ = poisson
    from paper_2305_19013_amd import ecg

    with pytest.raises(ecg.EcgError):
        _solve(torch, dev, p, restart=ora.RESTART_EVERY, restart_every=0)
    with pytest.raises(ecg.EcgError):
        _solve(torch, dev, p, restart=5)


def test_fp32_refined_with_restarts_reaches_fp64_accuracy(torch_dev, poisson):
    """Restarts inside the FP32 form's inner solves (iteration numbers are those of the inner
    solve): the refined solution reaches the FP64 true residual 1e-8."""
    torch, dev = torch_dev
    p, A = poisson
    rep, x, _ = _solve(torch, dev, p, tol=1e-8, precision=1, inner_tol=1e-4, replace_every=25,
                       restart=ora.RESTART_TOL, restart_tol=1e-3)
    assert rep["status"] == "ok" and rep["n_restart"] >= 1
    assert ora.true_relres(A, p.b, x) <= 1.01e-8
