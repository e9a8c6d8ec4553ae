"""GPU checks at the full sizes of the workloads, in the launch configurations the benchmark
times, against what the oracle (or SciPy) can compute at that size: sampled rows of the
products, the first iterations of the solve, and the true residual of whole solves.

Tolerances: sampled SpMM rows to 16 u sum |a||x| (u of the arithmetic); iterates to 1e-10
relative (FP64 parity bar); whole solves to a true relative residual of 1e-8 recomputed on
the host in FP64.
"""

import numpy as np
import pytest

import workloads as W
from oracle import ecg as ora

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_2305_19013_amd import ecg

    ecg.lib()
    return torch, torch.device("cuda:0")


class _Progress:
    """A @ X that prints a line every few products: a long oracle run keeps reporting."""

    def __init__(self, A):
        self.A, self.shape, self.count = A, A.shape, 0

    def __matmul__(self, X):
        self.count += 1
        if self.count % 4 == 0:
            print(f"  oracle: {self.count} products with A", flush=True)
        return self.A @ X


@pytest.fixture(scope="module")
def aniso():
    p = W.config("aniso3d128")  # n = 2,097,152, t = 32
    return p, p.A.to_scipy()


@pytest.mark.parametrize("t", [16, 32])
def test_spmm_full_size_sampled_rows(torch_dev, aniso, t):
    """Y = A X on the full 128^3 operator (diagonal-form kernel), 2000 sampled rows."""
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    p, A = aniso
    rng = np.random.default_rng(t)
    X = rng.standard_normal((p.n, t))
    Xt = torch.from_numpy(X).to(dev)
    Yt = torch.empty_like(Xt)
    ecg.debug_spmm(ecg.Operator.from_csr(p.A), t, Xt, Yt)
    rows = np.sort(rng.choice(p.n, 2000, replace=False))
    rows = np.r_[0, 1, p.n - 1, rows]  # include boundary rows
    Y = Yt[torch.from_numpy(rows).to(dev)].cpu().numpy()
    ref = A[rows] @ X
    bound = 16 * 2.0 ** -53 * (abs(A[rows]) @ np.abs(X))
    assert np.all(np.abs(Y - ref) <= bound + 1e-300)


def test_first_iterations_full_size_match_oracle(torch_dev, aniso):
    """The bench's FP64 step (aniso3d128, t = 32) stopped after 3 iterations."""
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    p, A = aniso
    ref = ora.flexible_sre_cg2(A, p.b, p.part, p.t, tol=p.tol, kmax=4, reduce=p.reduce, switch_tol=p.switch_tol,
                               t_min=p.t_min)
    op = ecg.Operator.from_csr(p.A)
    P = ecg.Partition(p.part, p.t)
    bt = torch.from_numpy(p.b).to(dev)
    xt = torch.zeros_like(bt)
    rep, rh = ecg.solve(op, P, bt, xt, ecg.options(tol=p.tol, kmax=4, reduce=p.reduce, switch_tol=p.switch_tol,
                                                   t_min=p.t_min, q_budget_bytes=4 * p.t * p.n * 8), rho_hist=True)
    assert rep["iters"] == ref.it == 3
    x = xt.cpu().numpy()
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    emax = np.abs(x - ref.x).max() / np.abs(ref.x).max()  # largest entry error
    assert err <= 1e-10 and emax <= 1e-10, (err, emax)
    assert np.abs(rh - np.array(ref.rho)).max() <= 1e-10 * ref.rho[0]


@pytest.mark.timeout(900)
def test_switch_window_full_size_matches_oracle(torch_dev, aniso):
    """The bench's FP64 step (aniso3d128, t = 32) for 12 iterations with the width halved at
    iteration 6 (scheduled): the CGS2 sweeps then run over stored blocks of widths 32 and 16
    (two spans) with a 16-wide candidate, at n = 2,097,152.  Iterates to 1e-10 (2-norm and
    largest entry), the recursive residual history entry by entry to 1e-10 rho_0."""
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    p, A = aniso
    kw = dict(reduce=ora.REDUCE_SCHEDULE, schedule=[6], t_min=16)
    print("oracle: aniso3d128 t=32, 12 iterations, halving at 6", flush=True)
    ref = ora.flexible_sre_cg2(_Progress(A), p.b, p.part, p.t, tol=p.tol, kmax=13, **kw)
    op = ecg.Operator.from_csr(p.A)
    P = ecg.Partition(p.part, p.t)
    bt = torch.from_numpy(p.b).to(dev)
    xt = torch.zeros_like(bt)
    rep, rh = ecg.solve(op, P, bt, xt, ecg.options(tol=p.tol, kmax=13, q_budget_bytes=16 * p.t * p.n * 8, **kw),
                        rho_hist=True)
    assert rep["iters"] == ref.it == 12 and rep["switch_iters"] == ref.switch_iters == [6]
    assert rep["vectors_stored"] == ref.mem == 5 * 32 + 7 * 16
    x = xt.cpu().numpy()
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    emax = np.abs(x - ref.x).max() / np.abs(ref.x).max()
    print(f"x_12: rel err {err:.2e}, largest entry err {emax:.2e}", flush=True)
    assert err <= 1e-10 and emax <= 1e-10
    assert np.abs(rh - np.array(ref.rho)).max() <= 1e-10 * ref.rho[0]


@pytest.mark.parametrize("t,its", [(16, 2), (64, 1)])
def test_aniso_other_widths_full_size_match_oracle(torch_dev, t, its):
    """aniso3d128 with t = 16 and t = 64 (2x2x4 and 2x2x16 boxes) at full size: the first
    iterations (two at t = 16 including a CGS2 sweep, one at t = 64)."""
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    p = W.config("aniso3d128", t=t)
    A = p.A.to_scipy()
    ref = ora.flexible_sre_cg2(A, p.b, p.part, p.t, tol=p.tol, kmax=its + 1)
    op = ecg.Operator.from_csr(p.A)
    P = ecg.Partition(p.part, p.t)
    bt = torch.from_numpy(p.b).to(dev)
    xt = torch.zeros_like(bt)
    rep, _ = ecg.solve(op, P, bt, xt, ecg.options(tol=p.tol, kmax=its + 1, q_budget_bytes=3 * p.t * p.n * 8))
    assert rep["iters"] == ref.it == its
    x = xt.cpu().numpy()
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    emax = np.abs(x - ref.x).max() / np.abs(ref.x).max()  # largest entry error
    assert err <= 1e-10 and emax <= 1e-10, (err, emax)


def test_jump3d160_full_size_with_halving_matches_oracle(torch_dev):
    """jump3d160 at full size (n = 4,096,000, t = 64 from 4x4x4 boxes): two iterations, the
    width halved to 32 at the second (scheduled), on the merged boxes."""
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    p = W.config("jump3d160")
    A = p.A.to_scipy()
    kw = dict(reduce=ora.REDUCE_SCHEDULE, schedule=[2], t_min=8)
    ref = ora.flexible_sre_cg2(A, p.b, p.part, p.t, tol=p.tol, kmax=3, **kw)
    op = ecg.Operator.from_csr(p.A)
    P = ecg.Partition(p.part, p.t)
    bt = torch.from_numpy(p.b).to(dev)
    xt = torch.zeros_like(bt)
    rep, rh = ecg.solve(op, P, bt, xt, ecg.options(tol=p.tol, kmax=3, q_budget_bytes=3 * p.t * p.n * 8, **kw),
                        rho_hist=True)
    assert rep["iters"] == ref.it == 2 and rep["switch_iters"] == [2] and rep["t_final"] == 32
    assert rep["vectors_stored"] == ref.mem
    x = xt.cpu().numpy()
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    emax = np.abs(x - ref.x).max() / np.abs(ref.x).max()  # largest entry error
    assert err <= 1e-10 and emax <= 1e-10, (err, emax)
    assert np.abs(rh - np.array(ref.rho)).max() <= 1e-10 * ref.rho[0]


@pytest.mark.parametrize("kind", ["bj_ic0", "chol64"])
def test_jump2d512_full_size_solves_to_tolerance(torch_dev, kind):
    """The metric's own 512^2 jumping-coefficient configuration (t = 32, one halving at
    switchTol 1e-5), block-Jacobi preconditioned as in the benchmark: the FP64 true
    residual recomputed on the host is <= 1e-8 and matches the reported one."""
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    p = W.config("jump2d512")
    A = p.A.to_scipy()
    op = ecg.Operator.from_csr(p.A)
    P = ecg.Partition(p.part, p.t)
    if kind == "bj_ic0":
        M = ecg.Precond.bj_ic0(op, P)
    else:
        M = ecg.Precond.bj(op, W.box_partition(p.grid, (8, 8)), ecg.BJ_CHOL)
    bt = torch.from_numpy(p.b).to(dev)
    xt = torch.zeros_like(bt)
    rep, _ = ecg.solve(op, P, bt, xt, ecg.options(tol=p.tol, reduce=p.reduce, switch_tol=p.switch_tol,
                                                  t_min=p.t_min, M=M, q_budget_bytes=400 * p.t * p.n * 8))
    assert rep["status"] == "ok" and len(rep["switch_iters"]) == 1
    x = xt.cpu().numpy()
    rel = ora.true_relres(A, p.b, x)
    assert rel <= 1.01e-8 and abs(rel - rep["relres_true"]) <= 1e-3 * rel
