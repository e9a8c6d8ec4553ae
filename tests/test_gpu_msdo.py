"""GPU parity of the MSDO-CG variants (Section 2.2; Algorithms 2, 4, 5) and of the
deflation reference against the FP64 oracle.

Same bar as the SRE-CG2 parity tests: iterates and residual histories to 1e-10 relative,
iteration counts, switch iterations, stored-vector and deflated-column counts exactly.
"""

import numpy as np
import pytest

import workloads as W
from oracle import ecg as ora
from oracle import precond as opre

pytestmark = pytest.mark.gpu


def _assert_x_close(x, xo, tol=1e-10):
    """Solution parity: relative 2-norm error and largest entry error (relative to the largest
    oracle entry) both within tol."""
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    emax = np.abs(x - xo).max() / np.abs(xo).max()
    assert err <= tol and emax <= tol, (err, emax)

MSDO, MODIFIED = 1, 2


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_2305_19013_amd import ecg

    ecg.lib()
    return torch, torch.device("cuda:0")


def _solve(torch, dev, csr, b, part, t, M=None, **kw):
    from paper_2305_19013_amd import ecg

    op = ecg.Operator.from_csr(csr)
    P = ecg.Partition(part, t)
    bt = torch.from_numpy(np.ascontiguousarray(b)).to(dev)
    xt = torch.zeros_like(bt)
    if M is not None:
        kw["M"] = M(ecg, op, P)
    rep, rh = ecg.solve(op, P, bt, xt, ecg.options(**kw), rho_hist=True)
    torch.cuda.synchronize()
    return rep, xt.cpu().numpy(), rh


def _same(rep, x, rh, ref):
    assert rep["iters"] == ref.it, (rep["iters"], ref.it)
    assert rep["switch_iters"] == ref.switch_iters
    assert rep["vectors_stored"] == ref.mem
    assert rep["deflated_cols"] == ref.deflated
    assert np.abs(rh - np.array(ref.rho)).max() <= 1e-10 * ref.rho[0]
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    emax = np.abs(x - ref.x).max() / np.abs(ref.x).max()  # largest entry error
    assert err <= 1e-10 and emax <= 1e-10, (err, emax)


def test_msdo_poisson64_parity(torch_dev):
    torch, dev = torch_dev
    p = W.config("poisson64")
    A = p.A.to_scipy()
    ref = ora.flexible_msdo_cg(A, p.b, p.part, p.t, tol=p.tol)
    rep, x, rh = _solve(torch, dev, p.A, p.b, p.part, p.t, tol=p.tol, variant=MSDO)
    assert rep["status"] == "ok"
    _same(rep, x, rh, ref)


def test_flexible_msdo_switch_parity(torch_dev):
    torch, dev = torch_dev
    p = W.config("poisson64")
    A = p.A.to_scipy()
    kw = dict(reduce=ora.REDUCE_ONCE, switch_tol=1e-4, t_min=2)
    ref = ora.flexible_msdo_cg(A, p.b, p.part, p.t, tol=p.tol, **kw)
    assert len(ref.switch_iters) == 1
    rep, x, rh = _solve(torch, dev, p.A, p.b, p.part, p.t, tol=p.tol, variant=MSDO, **kw)
    _same(rep, x, rh, ref)
    assert rep["vectors_stored"] == ora.memory_formula(p.t, ref.it, ref.sit)


def test_modified_msdo_parity(torch_dev):
    torch, dev = torch_dev
    p = W.config("poisson64")
    A = p.A.to_scipy()
    kw = dict(reduce=ora.REDUCE_ONCE, switch_tol=1e-4, t_min=2)
    ref = ora.flexible_sre_cg2(A, p.b, p.part, p.t, tol=p.tol, candidate="modified-msdo", **kw)
    rep, x, rh = _solve(torch, dev, p.A, p.b, p.part, p.t, tol=p.tol, variant=MODIFIED, **kw)
    _same(rep, x, rh, ref)


def test_msdo_block_jacobi_parity(torch_dev):
    """Algorithm 5: beta from M^{-1} r, split term L^{-T} T(L^{-1} r)."""
    torch, dev = torch_dev
    p = W.config("learn2d256", seed=11, scale=4)
    A = p.A.to_scipy()
    pre, _ = opre.bj_ic0_preconditioner(A, p.part)
    ref = ora.flexible_msdo_cg(A, p.b, p.part, p.t, tol=1e-8, precond=pre)
    rep, x, rh = _solve(torch, dev, p.A, p.b, p.part, p.t, tol=1e-8, variant=MSDO,
                        M=lambda ecg, op, P: ecg.Precond.bj_ic0(op, P))
    assert rep["iters"] == ref.it and rep["deflated_cols"] == ref.deflated
    _assert_x_close(x, ref.x)


def test_msdo_repeated_halving_parity(torch_dev):
    torch, dev = torch_dev
    p = W.config("jump3d160", scale=8)  # 20^3 grid, t = 64
    A = p.A.to_scipy()
    kw = dict(reduce=ora.REDUCE_SCHEDULE, schedule=[3, 5, 9], t_min=8)
    ref = ora.flexible_msdo_cg(A, p.b, p.part, p.t, tol=1e-30, kmax=13, **kw)
    rep, x, rh = _solve(torch, dev, p.A, p.b, p.part, p.t, tol=1e-30, kmax=13, variant=MSDO, **kw)
    assert rep["switch_iters"] == [3, 5, 9] and rep["t_final"] == 8
    _same(rep, x, rh, ref)


@pytest.mark.parametrize("n,t", [(48, 4), (45, 5), (60, 6)])
def test_deflation_reference_near_termination(torch_dev, n, t):
    """Past exact termination (iteration n/t + 1) the candidate's remainder after the
    A-orthonormalisation is rounding noise; measured against the norms before it, every
    column is dropped and both sides stop with a breakdown after storing n vectors."""
    torch, dev = torch_dev
    A = W.random_spd(n, 30.0, 17)
    b = W.rhs_uniform(n, 18)
    part = W.random_partition(n, t, 19)
    ref = ora.flexible_sre_cg2(A, b, part, t, tol=1e-30, kmax=n // t + 4)
    assert ref.status == "breakdown" and ref.mem == n
    rep, x, rh = _solve(torch, dev, W.dense_to_csr(A), b, part, t, tol=1e-30, kmax=n // t + 4)
    assert rep["status"] == "breakdown"
    assert rep["iters"] == ref.it and rep["deflated_cols"] == ref.deflated
    assert rep["vectors_stored"] == ref.mem <= n
    _assert_x_close(x, ref.x)


def test_variant_rejected(torch_dev):
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    p = W.config("poisson64")
    with pytest.raises(ecg.EcgError):
        _solve(torch, dev, p.A, p.b, p.part, p.t, variant=7)


def test_truncated_msdo_and_modified_msdo_parity(torch_dev):
    """Truncation (Section 3) applies to MSDO-CG and modified MSDO-CG as to SRE-CG2: Q is the
    last trunc blocks."""
    torch, dev = torch_dev
    p = W.config("poisson64")
    A = p.A.to_scipy()
    ref = ora.flexible_msdo_cg(A, p.b, p.part, p.t, tol=p.tol, trunc=6)
    rep, x, rh = _solve(torch, dev, p.A, p.b, p.part, p.t, tol=p.tol, variant=MSDO, trunc=6)
    assert rep["iters"] == ref.it and rep["trunc_used"] == 6
    _assert_x_close(x, ref.x)
    ref = ora.flexible_sre_cg2(A, p.b, p.part, p.t, tol=p.tol, trunc=2, candidate="modified-msdo")
    rep, x, rh = _solve(torch, dev, p.A, p.b, p.part, p.t, tol=p.tol, variant=MODIFIED, trunc=2)
    assert rep["iters"] == ref.it
    _assert_x_close(x, ref.x)
