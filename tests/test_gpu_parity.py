"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 iterates agree to 1e-10 relative (||x_gpu - x_ora|| <= 1e-10 ||x_ora||),
recursive residual norms to 1e-10 * rho_0, iteration counts, switch iterations and
stored-vector counts exactly.  Kernel building blocks agree with NumPy/SciPy products
to a few ulps of the accumulated magnitudes.
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


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_2305_19013_amd import ecg

    ecg.lib()  # raises if libecg.so is missing: no fallback
    return torch, torch.device("cuda:0")


def _t(torch, dev, a, dtype=None):
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a).to(dev) if dtype is None else torch.from_numpy(a).to(dev, dtype)


def _solve(torch, dev, csr, b, part, t, x0=None, **kw):
    from paper_2305_19013_amd import ecg

    op = ecg.Operator.from_csr(csr)
    P = ecg.Partition(part, t)
    bt = _t(torch, dev, b)
    xt = torch.zeros_like(bt) if x0 is None else _t(torch, dev, x0)
    hist = kw.pop("rho_hist", False)
    rep, rh = ecg.solve(op, P, bt, xt, ecg.options(**kw), rho_hist=hist)
    torch.cuda.synchronize()
    return rep, xt.cpu().numpy(), rh


# ---------------------------------------------------------------- building blocks
@pytest.mark.parametrize("t", [1, 8, 32, 64])
@pytest.mark.parametrize("kind", ["uniform", "ragged"])
def test_spmm_general_csr_matches_scipy(torch_dev, t, kind):
    """Matrices with scattered columns (more than 16 distinct diagonals): the SELL-C-sigma
    kernel the solver picks and the CSR kernel agree bitwise, and both hold the dot-product
    bound against SciPy.  "ragged": row lengths from 1 to ~300 (a few dense rows), n not a
    multiple of the 64-row slice, so the sorted windows and the slice padding matter."""
    torch, dev = torch_dev
    import scipy.sparse as sp

    from paper_2305_19013_amd import ecg

    n = 5003
    rng = np.random.default_rng(40 + t)
    R = sp.random(n, n, density=6.0 / n, random_state=rng, format="csr")
    if kind == "ragged":
        dense = sp.csr_matrix((rng.standard_normal((7, n)) * (rng.random((7, n)) < 0.06)))
        rows = sp.csr_matrix((np.ones(7), (rng.choice(n, 7, replace=False), np.arange(7))), shape=(n, 7))
        R = R + rows @ dense
    A = sp.csr_matrix(R + R.T + sp.eye(n) * 10.0)
    A.sort_indices()
    csr = W.CSR(n, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64))
    X = rng.standard_normal((n, t))
    Xt = _t(torch, dev, X)
    op = ecg.Operator.from_csr(csr)
    Ys = {}
    for k in (ecg.SPMM_AUTO, ecg.SPMM_SELL, ecg.SPMM_CSR):
        Yt = torch.full_like(Xt, np.nan)
        ecg.debug_spmm_kernel(op, k, t, Xt, Yt)
        Ys[k] = Yt.cpu().numpy()
    assert np.array_equal(Ys[ecg.SPMM_SELL], Ys[ecg.SPMM_CSR]) and np.array_equal(Ys[ecg.SPMM_AUTO], Ys[ecg.SPMM_SELL])
    scale = abs(A) @ np.abs(X)
    assert np.all(np.abs(Ys[ecg.SPMM_SELL] - A @ X) <= 2.0 ** -53 * 16 * scale + 1e-300)


@pytest.mark.parametrize("t", [1, 8, 32, 64])
def test_spmm_matches_scipy(torch_dev, t):
    """A 5-point operator (5 diagonals): the diagonal-form kernel."""
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    p = W.config("jump2d512", scale=8)
    A = p.A.to_scipy()
    X = np.random.default_rng(t).standard_normal((p.n, t))
    op = ecg.Operator.from_csr(p.A)
    Xt = _t(torch, dev, X)
    Yt = torch.empty_like(Xt)
    ecg.debug_spmm(op, t, Xt, Yt)
    ref = A @ X
    scale = abs(A) @ np.abs(X)
    assert np.all(np.abs(Yt.cpu().numpy() - ref) <= 4e-16 * 8 * scale + 1e-300)


@pytest.mark.parametrize("level", [0, 1, 2])
def test_split_is_exact(torch_dev, level):
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    p = W.config("jump2d512", scale=8)
    P = ecg.Partition(p.part, p.t)
    v = W.rhs_uniform(p.n, 5)
    tl = p.t >> level
    out = torch.empty((p.n, tl), dtype=torch.float64, device=dev)
    ecg.debug_split(P, level, _t(torch, dev, v), out)
    assert np.array_equal(out.cpu().numpy(), ora.split(v, ora.merged_partition(p.part, level), tl))


GRAM_CASES = [(4099, 3, 8, 8), (4099, 2, 32, 16), (70001, 5, 32, 32), (3000, 1, 64, 64), (1027, 4, 16, 64),
              (5000, 3, 64, 8), (1027, 3, 16, 32), (4099, 5, 16, 16), (2053, 7, 32, 32), (777, 1, 16, 16),
              # 8-wide candidates and stored blocks (after halvings): pairs of 8-column blocks,
              # an odd count of them, a single one, and 8-wide candidates against wider blocks
              (1027, 7, 8, 8), (777, 1, 8, 8), (70001, 9, 8, 8), (4099, 5, 16, 8), (2053, 2, 32, 8)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,nb,wq,t", GRAM_CASES)
def test_gram_and_update_match_numpy(torch_dev, n, nb, wq, t, dtype):
    """Blocks narrower than a 16-byte lane load are read in groups (FP64 width 16, FP32
    widths 16 and 32), including groups cut short by the end of the span.  Bounds: the
    standard dot-product error bound, gamma_K sum |a||b| with unit roundoff u of the type."""
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    u = 2.0 ** -53 if dtype == "f64" else 2.0 ** -24
    npt = np.float64 if dtype == "f64" else np.float32
    tt = torch.float64 if dtype == "f64" else torch.float32
    rng = np.random.default_rng(n + t)
    Q = rng.standard_normal((nb, n, wq)).astype(npt)
    Y = rng.standard_normal((n, t)).astype(npt)
    Qm = np.concatenate([Q[j] for j in range(nb)], axis=1).astype(np.float64)  # n x (nb*wq)
    Qt = torch.from_numpy(Q).to(dev)
    Yt = torch.from_numpy(Y).to(dev)
    Gt = torch.empty((nb * wq, t), dtype=tt, device=dev)
    ecg.debug_gram(n, nb, wq, Qt, t, Yt, Gt)
    G = Gt.cpu().numpy().astype(np.float64)
    ref = Qm.T @ Y.astype(np.float64)
    bound = 2 * n * u * (np.abs(Qm).T @ np.abs(Y.astype(np.float64))) + 1e-30
    assert np.all(np.abs(G - ref) <= bound)
    W0 = rng.standard_normal((n, t)).astype(npt)
    Wt = torch.from_numpy(W0).to(dev)
    ecg.debug_update(n, nb, wq, Qt, t, Gt, Wt)
    Gq = Gt.cpu().numpy().astype(np.float64)
    refw = W0.astype(np.float64) - Qm @ Gq
    boundw = 2 * (nb * wq + 1) * u * (np.abs(W0.astype(np.float64)) + np.abs(Qm) @ np.abs(Gq)) + 1e-30
    assert np.all(np.abs(Wt.cpu().numpy().astype(np.float64) - refw) <= boundw)


def test_block_jacobi_ic0_apply_matches_oracle(torch_dev):
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    p = W.config("learn2d256", seed=7, scale=4)
    A = p.A.to_scipy()
    _, L = opre.bj_ic0_preconditioner(A, p.part)
    op = ecg.Operator.from_csr(p.A)
    P = ecg.Partition(p.part, p.t)
    M = ecg.Precond.bj_ic0(op, P)
    X = np.random.default_rng(1).standard_normal((p.n, 16))
    Xt = _t(torch, dev, X)
    Yt = torch.empty_like(Xt)
    import scipy.sparse.linalg as spl

    M.apply(0, 16, Xt, Yt)
    ref = spl.spsolve_triangular(L.tocsr(), X, lower=True)
    assert np.abs(Yt.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    M.apply(1, 16, Xt, Yt)
    ref = spl.spsolve_triangular(L.T.tocsr(), X, lower=False)
    assert np.abs(Yt.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


# ---------------------------------------------------------------- whole solves
def _check_iterates(torch, dev, csr, b, part, t, ref, ks, **kw):
    """GPU solves stopped after k iterations (kmax = k + 1) against oracle iterates."""
    for k in ks:
        rep, x, _ = _solve(torch, dev, csr, b, part, t, kmax=k + 1, **kw)
        assert rep["iters"] == k
        xo = ref.iterates[k - 1]
        err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
        assert err <= 1e-10, (k, err)


def test_poisson64_parity(torch_dev):
    """The 64x64 Poisson workload (t = 8, 2x4 boxes, no reduction)."""
    torch, dev = torch_dev
    p = W.config("poisson64")
    A = p.A.to_scipy()
    ref = ora.flexible_sre_cg2(A, p.b, p.part, p.t, tol=p.tol, record=True)
    rep, x, rh = _solve(torch, dev, p.A, p.b, p.part, p.t, tol=p.tol, rho_hist=True)
    assert rep["status"] == "ok"
    assert rep["iters"] == ref.it and rep["vectors_stored"] == ref.mem
    assert np.abs(rh - np.array(ref.rho)).max() <= 1e-10 * ref.rho[0]
    _assert_x_close(x, ref.x)
    assert rep["relres_true"] <= 1.01e-8
    _check_iterates(torch, dev, p.A, p.b, p.part, p.t, ref, [1, 2, 5, 20, 60], tol=p.tol)


def test_poisson64_flexible_switch_parity(torch_dev):
    torch, dev = torch_dev
    p = W.config("poisson64")
    A = p.A.to_scipy()
    kw = dict(reduce=ora.REDUCE_ONCE, switch_tol=1e-4, t_min=2)
    ref = ora.flexible_sre_cg2(A, p.b, p.part, p.t, tol=p.tol, record=True, **kw)
    assert len(ref.switch_iters) == 1
    rep, x, rh = _solve(torch, dev, p.A, p.b, p.part, p.t, tol=p.tol, rho_hist=True, **kw)
    assert rep["iters"] == ref.it and rep["switch_iters"] == ref.switch_iters
    assert rep["vectors_stored"] == ref.mem == ora.memory_formula(p.t, ref.it, ref.sit)
    assert np.abs(rh - np.array(ref.rho)).max() <= 1e-10 * ref.rho[0]
    s = ref.switch_iters[0]
    _check_iterates(torch, dev, p.A, p.b, p.part, p.t, ref, [s - 1, s, s + 3, ref.it], tol=p.tol, **kw)


def test_repeated_halving_and_schedule_parity(torch_dev):
    torch, dev = torch_dev
    p = W.config("jump3d160", scale=8)  # 20^3 grid, t = 64 from 4x4x4 boxes
    A = p.A.to_scipy()
    kw = dict(reduce=ora.REDUCE_SCHEDULE, schedule=[3, 5, 9], t_min=8)
    ref = ora.flexible_sre_cg2(A, p.b, p.part, p.t, tol=1e-30, kmax=13, record=True, **kw)
    rep, x, _ = _solve(torch, dev, p.A, p.b, p.part, p.t, tol=1e-30, kmax=13, **kw)
    assert rep["switch_iters"] == [3, 5, 9] and rep["t_final"] == 8
    assert rep["iters"] == 12 and rep["vectors_stored"] == ref.mem
    _assert_x_close(x, ref.x)


@pytest.mark.parametrize("n,t", [(48, 4), (45, 5), (50, 4), (60, 6)])
def test_tiny_dense_termination_and_padding(torch_dev, n, t):
    """Ragged widths (t padded to a power of two inside) and exact termination."""
    torch, dev = torch_dev
    A = W.random_spd(n, 30.0, 17)
    b = W.rhs_uniform(n, 18)
    part = W.random_partition(n, t, 19)
    ref = ora.flexible_sre_cg2(A, b, part, t, tol=1e-11, record=True)
    rep, x, _ = _solve(torch, dev, W.dense_to_csr(A), b, part, t, tol=1e-11)
    assert rep["iters"] == ref.it == -(-n // t)
    assert rep["vectors_stored"] == ref.mem == n
    assert rep["deflated_cols"] == ref.deflated
    _assert_x_close(x, ref.x)


def test_deflated_zero_subdomain(torch_dev):
    torch, dev = torch_dev
    n, t = 40, 4
    A = W.random_spd(n, 50.0, 29)
    b = W.rhs_uniform(n, 30)
    part = W.random_partition(n, t, 31)
    b[part == 2] = 0.0
    ref = ora.flexible_sre_cg2(A, b, part, t, tol=1e-10, record=True)
    rep, x, _ = _solve(torch, dev, W.dense_to_csr(A), b, part, t, tol=1e-10)
    assert ref.widths[0] == 3
    assert rep["iters"] == ref.it and rep["vectors_stored"] == ref.mem and rep["deflated_cols"] == ref.deflated
    _assert_x_close(x, ref.x)
    rep2, _, _ = _solve(torch, dev, W.dense_to_csr(A), b, part, t, tol=1e-10, deflate_tol=-1.0)
    assert rep2["status"] == "breakdown"


def test_kmax_not_converged(torch_dev):
    torch, dev = torch_dev
    p = W.config("poisson64")
    rep, _, _ = _solve(torch, dev, p.A, p.b, p.part, p.t, kmax=3)
    assert rep["status"] == "not_converged" and rep["iters"] == 2


def test_q_budget_truncation_parity(torch_dev):
    """A Q budget of 6 blocks = truncated SRE-CG2 with trunc = 6 (Section 3)."""
    torch, dev = torch_dev
    p = W.config("poisson64")
    A = p.A.to_scipy()
    ref = ora.flexible_sre_cg2(A, p.b, p.part, p.t, tol=p.tol, trunc=6)
    rep, x, _ = _solve(torch, dev, p.A, p.b, p.part, p.t, tol=p.tol, q_budget_bytes=6 * p.n * 8 * 8)
    assert rep["iters"] == ref.it
    _assert_x_close(x, ref.x)
    rep2, x2, _ = _solve(torch, dev, p.A, p.b, p.part, p.t, tol=p.tol, trunc=6)
    assert rep2["iters"] == ref.it
    _assert_x_close(x2, ref.x)


def test_nonzero_initial_guess(torch_dev):
    torch, dev = torch_dev
    p = W.config("poisson64")
    A = p.A.to_scipy()
    x0 = W.rhs_uniform(p.n, 77)
    ref = ora.flexible_sre_cg2(A, p.b, p.part, p.t, x0=x0, tol=p.tol)
    rep, x, _ = _solve(torch, dev, p.A, p.b, p.part, p.t, x0=x0, tol=p.tol)
    assert rep["iters"] == ref.it
    _assert_x_close(x, ref.x)


def test_block_jacobi_preconditioned_parity(torch_dev):
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    p = W.config("learn2d256", seed=11, scale=4)  # 64x64, t = 16
    A = p.A.to_scipy()
    pre, _ = opre.bj_ic0_preconditioner(A, p.part)
    ref = ora.flexible_sre_cg2(A, p.b, p.part, p.t, tol=1e-8, precond=pre, record=True)
    op = ecg.Operator.from_csr(p.A)
    P = ecg.Partition(p.part, p.t)
    M = ecg.Precond.bj_ic0(op, P)
    bt = _t(torch, dev, p.b)
    xt = torch.zeros_like(bt)
    rep, _ = ecg.solve(op, P, bt, xt, ecg.options(tol=1e-8, M=M))
    assert rep["iters"] == ref.it
    x = xt.cpu().numpy()
    _assert_x_close(x, ref.x)


def test_factor_preconditioned_parity(torch_dev):
    """M^{-1} = G G^T with G = D^{-1/2} + strictly lower part (a Jacobi-like factor)."""
    torch, dev = torch_dev
    import scipy.sparse as sp

    from paper_2305_19013_amd import ecg

    p = W.config("learn2d256", seed=12, scale=4)
    A = p.A.to_scipy()
    d = A.diagonal()
    low = sp.tril(A, -1, format="csr")
    G = sp.csr_matrix(sp.diags(1.0 / np.sqrt(d)) - 0.3 * sp.diags(1.0 / d) @ low @ sp.diags(1.0 / np.sqrt(d)))
    G = sp.csr_matrix(sp.tril(G))
    G.sort_indices()
    pre = opre.factor_preconditioner(G)
    ref = ora.flexible_sre_cg2(A, p.b, p.part, p.t, tol=1e-8, precond=pre, reduce=ora.REDUCE_ONCE,
                               switch_tol=1e-4, t_min=2)
    M = ecg.Precond.factor(G.indptr, G.indices, G.data)
    rep, x, _ = _solve(torch, dev, p.A, p.b, p.part, p.t, tol=1e-8, M=M, reduce=ora.REDUCE_ONCE,
                       switch_tol=1e-4, t_min=2)
    assert rep["iters"] == ref.it and rep["switch_iters"] == ref.switch_iters
    _assert_x_close(x, ref.x)


def test_fp32_refined_reaches_fp64_accuracy(torch_dev):
    torch, dev = torch_dev
    p = W.config("poisson64")
    A = p.A.to_scipy()
    rep, x, _ = _solve(torch, dev, p.A, p.b, p.part, p.t, tol=1e-8, precision=1, inner_tol=1e-4,
                       replace_every=25)
    assert rep["status"] == "ok"
    assert rep["relres_true"] <= 1e-8
    assert ora.true_relres(A, p.b, x) <= 1e-8
    xs = __import__("scipy.sparse.linalg", fromlist=["spsolve"]).spsolve(A.tocsc(), p.b)
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)


@pytest.mark.parametrize("case", ["poisson64", "jump2d256_chol64"])
def test_fp32_refined_error_against_oracle(torch_dev, case):
    """The FP32 form's solution against the FP64 oracle's on configurations the oracle
    finishes: 64x64 Poisson (t = 8) and the 256x256 jumping-coefficient operator (t = 32 with
    one halving) under block-Jacobi Cholesky on 64 blocks.  Both solutions have a true
    relative residual <= 1e-8, so they differ by at most ||A^{-1}|| (||r_fp32|| + ||r_oracle||)
    = (relres_fp32 + relres_oracle) ||b|| / lambda_min(A); the measured error is reported and
    held to that bound."""
    torch, dev = torch_dev
    import scipy.sparse.linalg as spl

    from paper_2305_19013_amd import ecg

    if case == "poisson64":
        p = W.config("poisson64")
        kw, M, pre = {}, None, None
    else:
        p = W.config("jump2d512", scale=2)
        blocks = W.box_partition(p.grid, (8, 8))
        kw = dict(reduce=p.reduce, switch_tol=p.switch_tol, t_min=p.t_min)
        pre, _ = opre.bj_chol_preconditioner(p.A.to_scipy(), blocks)
    A = p.A.to_scipy()
    ref = ora.flexible_sre_cg2(A, p.b, p.part, p.t, tol=p.tol, precond=pre, **kw)
    op = ecg.Operator.from_csr(p.A)
    P = ecg.Partition(p.part, p.t)
    if pre is not None:
        M = ecg.Precond.bj(op, blocks, ecg.BJ_CHOL)
    bt = _t(torch, dev, p.b)
    xt = torch.zeros_like(bt)
    rep, _ = ecg.solve(op, P, bt, xt, ecg.options(tol=p.tol, precision=1, inner_tol=1e-4, replace_every=25, M=M,
                                                  **kw))
    torch.cuda.synchronize()
    x = xt.cpu().numpy()
    assert rep["status"] == "ok"
    rel32 = ora.true_relres(A, p.b, x)
    relo = ora.true_relres(A, p.b, ref.x)
    assert rel32 <= 1e-8 and relo <= 1.01e-8
    lmin = float(spl.eigsh(A, k=1, sigma=0, which="LM", return_eigenvectors=False)[0])
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    bound = (rel32 + relo) * np.linalg.norm(p.b) / lmin / np.linalg.norm(ref.x)
    print(f"{case}: FP32-refined vs oracle {err:.2e} (bound {bound:.2e}); iterations {rep['iters']} in "
          f"{rep['outer_iters']} steps vs oracle {ref.it}", flush=True)
    assert err <= bound


def test_determinism_bitwise(torch_dev):
    torch, dev = torch_dev
    p = W.config("jump2d512", scale=4)
    r1, x1, _ = _solve(torch, dev, p.A, p.b, p.part, p.t, kmax=40)
    r2, x2, _ = _solve(torch, dev, p.A, p.b, p.part, p.t, kmax=40)
    assert np.array_equal(x1, x2)


def test_zero_residual_returns_immediately(torch_dev):
    """b = 0 with x0 = 0: rho_0 = 0, no iteration, x stays zero (both precision forms)."""
    torch, dev = torch_dev
    p = W.config("poisson64")
    for precision in (0, 1):
        rep, x, _ = _solve(torch, dev, p.A, np.zeros(p.n), p.part, p.t, tol=p.tol, precision=precision)
        assert rep["status"] == "ok" and rep["iters"] == 0 and not np.any(x)


def test_invalid_inputs_rejected_before_device_work(torch_dev):
    """Partition values out of range, an empty subdomain, t > 64, NaN in b: ECG_EINVAL."""
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    p = W.config("poisson64")
    bad = p.part.copy()
    bad[0] = p.t  # out of range
    with pytest.raises(ecg.EcgError):
        ecg.Partition(bad, p.t)
    empty = p.part.copy()
    empty[empty == 3] = 2  # subdomain 3 empty
    with pytest.raises(ecg.EcgError):
        ecg.Partition(empty, p.t)
    with pytest.raises(ecg.EcgError):
        ecg.Partition(np.arange(p.n, dtype=np.int32) % 65, 65)
    b = p.b.copy()
    b[5] = np.nan
    with pytest.raises(ecg.EcgError):
        _solve(torch, dev, p.A, b, p.part, p.t, tol=p.tol)


@pytest.mark.parametrize("switch_tol,min_gap", [(1e-3, 5), (1e-2, 3)])
def test_repeat_rule_parity(torch_dev, switch_tol, min_gap):
    """Repeated halving on tol1 < switchTol, at least min_gap iterations apart, 8 -> 4 -> 2."""
    torch, dev = torch_dev
    p = W.config("poisson64")
    A = p.A.to_scipy()
    kw = dict(reduce=ora.REDUCE_REPEAT, switch_tol=switch_tol, t_min=2, min_gap=min_gap)
    ref = ora.flexible_sre_cg2(A, p.b, p.part, p.t, tol=p.tol, **kw)
    assert len(ref.switch_iters) == 2 and ref.t_final == 2
    rep, x, rh = _solve(torch, dev, p.A, p.b, p.part, p.t, tol=p.tol, rho_hist=True, **kw)
    assert rep["iters"] == ref.it and rep["switch_iters"] == ref.switch_iters and rep["t_final"] == 2
    assert rep["vectors_stored"] == ref.mem
    assert np.abs(rh - np.array(ref.rho)).max() <= 1e-10 * ref.rho[0]
    _assert_x_close(x, ref.x)


def test_spmv_info_and_kernel_statistics(torch_dev):
    """ecg_spmv (FP64 y = A x), ecg_operator_info, and the per-kernel statistics: a solve of k
    iterations records k final updates, and the byte counts are the stated algorithmic ones."""
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    p = W.config("poisson64")
    A = p.A.to_scipy()
    op = ecg.Operator.from_csr(p.A)
    assert op.info() == (p.n, p.A.nnz)
    x = np.random.default_rng(3).standard_normal(p.n)
    xt = _t(torch, dev, x)
    yt = torch.empty_like(xt)
    op.spmv(xt, yt)
    assert np.abs(yt.cpu().numpy() - A @ x).max() <= 1e-14 * np.abs(A @ x).max()
    ecg.stats_read(reset=True)
    ecg.stats_enable(True)
    rep, _, _ = _solve(torch, dev, p.A, p.b, p.part, p.t, tol=p.tol, kmax=11)
    ecg.stats_enable(False)
    st = ecg.stats_read(reset=True)
    assert rep["iters"] == 10
    assert st["final_update"]["count"] == 10 and st["final_update"]["ms"] > 0
    assert st["final_update"]["bytes"] == pytest.approx(10 * (4 * 8 * p.n * p.t + p.n * (2 * 8 + 2 * 8)))
    assert st["cgs2_gram"]["count"] == st["cgs2_update"]["count"] == 2 * 9  # two passes from k = 2 on


def test_solve_rejects_small_or_misaligned_workspace(torch_dev):
    """ecg_solve through the raw ABI: a workspace one byte short is ECG_ENOMEM, one not
    256-byte aligned is ECG_EINVAL; neither touches x."""
    torch, dev = torch_dev
    import ctypes as C

    from paper_2305_19013_amd import ecg

    p = W.config("poisson64")
    op = ecg.Operator.from_csr(p.A)
    P = ecg.Partition(p.part, p.t)
    o = ecg.options(tol=p.tol)
    need = ecg.workspace_size(op, P, o)
    ws = torch.empty(need + 512, dtype=torch.uint8, device=dev)
    b = _t(torch, dev, p.b)
    x = torch.full_like(b, 7.0)
    rep = ecg.Report()
    L = ecg.lib()
    base = ws.data_ptr()
    aligned = (base + 255) // 256 * 256
    st = L.ecg_solve(op.handle, P.handle, b.data_ptr(), x.data_ptr(), C.byref(o), aligned, need - 1,
                     ecg._stream(), C.byref(rep), None)
    assert st == -2 and "workspace" in L.ecg_last_error().decode()
    st = L.ecg_solve(op.handle, P.handle, b.data_ptr(), x.data_ptr(), C.byref(o), aligned + 8, need,
                     ecg._stream(), C.byref(rep), None)
    assert st == -1
    torch.cuda.synchronize()
    assert bool(torch.all(x == 7.0))


def test_mismatched_preconditioner_odd_halving_and_bad_tensors_rejected(torch_dev):
    """Host-side checks before any kernel: a band-Cholesky preconditioner built on another
    operator size, a halving of an odd width (subdomains merge in pairs, Section 4), and
    vectors that are not contiguous float64 device tensors of length n."""
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    p = W.config("poisson64")
    small = W.config("poisson64", scale=2)  # 32 x 32
    op_small = ecg.Operator.from_csr(small.A)
    M_small = ecg.Precond.bj(op_small, W.box_partition(small.grid, (4, 4)), ecg.BJ_CHOL)
    with pytest.raises(ecg.EcgError) as e:
        _solve(torch, dev, p.A, p.b, p.part, p.t, tol=p.tol, M=M_small)
    assert e.value.status == ecg.ECG_EINVAL
    n = 60
    A = W.random_spd(n, 30.0, 5)
    b = W.rhs_uniform(n, 6)
    for t, kw in ((5, dict(reduce=ora.REDUCE_ONCE, t_min=1)), (6, dict(reduce=ora.REDUCE_REPEAT, t_min=1)),
                  (6, dict(reduce=ora.REDUCE_SCHEDULE, schedule=[2, 4], t_min=1))):
        part = W.random_partition(n, t, 7)
        with pytest.raises(ecg.EcgError) as e:
            _solve(torch, dev, W.dense_to_csr(A), b, part, t, **kw)
        assert e.value.status == ecg.ECG_EINVAL
        with pytest.raises(ValueError):
            ora.flexible_sre_cg2(A, b, part, t, **kw)
    # 6 -> 3 is allowed when t_min stops the halving there
    part = W.random_partition(n, 6, 7)
    rep, _, _ = _solve(torch, dev, W.dense_to_csr(A), b, part, 6, reduce=ora.REDUCE_REPEAT, t_min=3)
    assert rep["status"] == "ok"
    op = ecg.Operator.from_csr(p.A)
    P = ecg.Partition(p.part, p.t)
    bt = _t(torch, dev, p.b)
    for bad in (bt.float(), bt[:-1], torch.zeros(2 * p.n, dtype=torch.float64, device=dev)[::2], bt.cpu()):
        with pytest.raises(ValueError):
            ecg.solve(op, P, bad, torch.zeros_like(bt), ecg.options(tol=p.tol))
