"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here re-types the oracle's own formulas: each check uses an
independent definition (50-digit subspace projections, dense direct solves,
LAPACK/CG references) or a property the paper states.
"""

import os

import numpy as np
import pytest

import workloads as W
from oracle import brute, ecg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def spl_solve(A, b):
    import scipy.sparse.linalg as spl

    return spl.spsolve(A.tocsc(), b)


def tiny(n=40, t=4, kappa=50.0, seed=1):
    A = W.random_spd(n, kappa, seed)
    b = W.rhs_uniform(n, seed + 1)
    part = W.random_partition(n, t, seed + 2)
    return A, b, part


# ---------------------------------------------------------------- split operator
def test_split_sums_back_and_is_disjoint():
    # T^t(v) 1_t = v (proof of Theorem 2) and one nonzero per row (eq. (Tt))
    rng = np.random.default_rng(0)
    v = rng.standard_normal(50)
    part = W.random_partition(50, 8, 1)
    T = ecg.split(v, part, 8)
    assert np.array_equal(T.sum(axis=1), v)
    assert np.all((T != 0).sum(axis=1) <= 1)
    for j in range(8):
        assert np.array_equal(T[part == j, j], v[part == j])


def test_halving_merges_consecutive_pairs():
    # delta-tilde_i = delta_{2i-1} U delta_{2i} (1-based) -> id >> 1 (0-based)
    part = np.arange(16, dtype=np.int32)
    merged = ecg.merged_partition(part, 1)
    assert list(merged) == [i // 2 for i in range(16)]
    rng = np.random.default_rng(3)
    v = rng.standard_normal(16)
    assert np.array_equal(ecg.split(v, merged, 8), ecg.split(v, part, 16).reshape(16, 8, 2).sum(axis=2))


def test_box_partition_halving_keeps_boxes():
    # Morton numbering: part >> 1 of a 4x8 box layout is the 4x4 box layout
    p8 = W.box_partition((64, 64), (4, 8))
    p4 = W.box_partition((64, 64), (4, 4))
    # same sets up to relabelling
    pairs = set(zip((p8 >> 1).tolist(), p4.tolist()))
    assert len(pairs) == 16
    assert len({a for a, _ in pairs}) == 16


# ---------------------------------------------------------------- iterates vs definitions
def test_iterates_equal_krylov_galerkin_projection():
    # x_k is the Galerkin iterate on x0 + K_{k,t}(A, r0) (Section 2), 50 digits
    A, b, part = tiny()
    res = ecg.flexible_sre_cg2(A, b, part, 4, tol=1e-14, record=True)
    for k in (1, 2, 4, 7):
        xk = brute.krylov_projection(A, b, part, 4, k)
        assert np.linalg.norm(res.iterates[k - 1] - xk) <= 1e-12 * np.linalg.norm(xk)


def test_flexible_iterates_equal_subspace_recursion():
    # with a switch at k=4: the subspaces Algorithm 3 builds, defined basis-free
    A, b, part = tiny(n=40, t=8, seed=5)
    res = ecg.flexible_sre_cg2(A, b, part, 8, tol=1e-14, reduce=ecg.REDUCE_SCHEDULE,
                               schedule=[4], t_min=1, record=True)
    assert res.switch_iters == [4]
    xs = brute.recursion_projection(A, b, part, 8, 6, [4])
    for k in range(6):
        assert np.linalg.norm(res.iterates[k] - xs[k]) <= 1e-12 * np.linalg.norm(xs[k])
    assert res.widths[:6] == [8, 8, 8, 4, 4, 4]


def test_t1_is_cg():
    # Theorem 2 with t = 1: the enlarged subspace is the Krylov subspace
    A, b, _ = tiny(n=30, t=1)
    part = np.zeros(30, dtype=np.int32)
    res = ecg.flexible_sre_cg2(A, b, part, 1, tol=1e-14, record=True)
    xs = brute.cg_iterates(A, b, 12)
    for k in range(12):
        assert np.linalg.norm(res.iterates[k] - xs[k]) <= 1e-11 * np.linalg.norm(xs[k])


def test_dense_direct_solve():
    A, b, part = tiny(n=48, t=6, kappa=1e3, seed=7)
    res = ecg.flexible_sre_cg2(A, b, part, 6, tol=1e-12)
    x = np.linalg.solve(A, b)
    assert res.status == "converged"
    assert np.linalg.norm(res.x - x) <= 1e-9 * np.linalg.norm(x)


# ---------------------------------------------------------------- Petrov-Galerkin invariants
def test_a_orthonormal_basis_and_galerkin_condition():
    A, b, part = tiny(n=64, t=4, kappa=1e3, seed=11)
    res = ecg.flexible_sre_cg2(A, b, part, 4, tol=1e-10, record=True)
    Q = np.hstack(res.blocks)
    assert np.abs(Q.T @ A @ Q - np.eye(Q.shape[1])).max() <= 1e-12
    for k in range(1, len(res.blocks) + 1):
        Qk = np.hstack(res.blocks[:k])
        rk = b - A @ res.iterates[k - 1]
        assert np.linalg.norm(Qk.T @ rk) <= 1e-12 * np.linalg.norm(b)
        # x_k - x_0 = Q_k Q_k^T r_0 (A-orthonormal basis of the search space)
        assert np.linalg.norm(res.iterates[k - 1] - Qk @ (Qk.T @ b)) <= 1e-11 * np.linalg.norm(res.iterates[k - 1])


def test_monotone_a_norm_error_and_not_worse_than_cg():
    # nested subspaces (Section 2) and K_k subset of K_{k,t} (Theorem 2)
    A, b, part = tiny(n=48, t=4, kappa=1e3, seed=13)
    xs = np.linalg.solve(A, b)
    res = ecg.flexible_sre_cg2(A, b, part, 4, tol=1e-12, record=True)
    _, _, cgit = ecg.cg(A, b, tol=1e-30, kmax=len(res.iterates), record=True)
    errs = [brute.a_norm_error(A, xs, x) for x in res.iterates]
    assert all(e2 <= e1 * (1 + 1e-10) for e1, e2 in zip(errs, errs[1:]))
    for k in range(len(res.iterates)):
        assert errs[k] <= brute.a_norm_error(A, xs, cgit[k]) * (1 + 1e-8) + 1e-12


@pytest.mark.parametrize("n,t", [(48, 4), (45, 5), (50, 4)])
def test_termination_in_ceil_n_over_t(n, t):
    # exact arithmetic + full rank: the subspace is all of R^n after ceil(n/t) blocks;
    # when t does not divide n the last block has dependent columns and is deflated
    A, b, part = tiny(n=n, t=t, kappa=30.0, seed=17)
    res = ecg.flexible_sre_cg2(A, b, part, t, tol=1e-11)
    assert res.status == "converged"
    assert res.it == -(-n // t)
    assert res.mem == n
    assert res.deflated == (t * res.it - n)


# ---------------------------------------------------------------- truncation (Section 3)
def test_truncation_two_blocks_matches_full_early():
    # Section 2.1: W_k = A W_{k-1} need only be A-orthonormalised against the two
    # previous blocks in exact arithmetic (SRE-CG = truncated SRE-CG2 with trunc = 2)
    A, b, part = tiny(n=60, t=4, kappa=20.0, seed=19)
    full = ecg.flexible_sre_cg2(A, b, part, 4, tol=1e-12, record=True)
    tr = ecg.flexible_sre_cg2(A, b, part, 4, tol=1e-12, trunc=2, record=True)
    for k in range(6):
        assert np.linalg.norm(full.iterates[k] - tr.iterates[k]) <= 1e-9 * np.linalg.norm(full.iterates[k])


# ---------------------------------------------------------------- memory bookkeeping
def _golden_rows():
    rows = []
    with open(os.path.join(GOLDEN, "paper_flex_sre_cg2.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            m, t, tol, it, sit, mem = line.split()
            rows.append((m, int(t), tol, int(it), int(sit), int(mem)))
    return rows


def test_memory_formula_reproduces_paper_tables():
    rows = _golden_rows()
    assert len(rows) == 96
    for m, t, tol, it, sit, mem in rows:
        assert ecg.memory_formula(t, it, sit) == mem, (m, t, tol)


def _restart_rows():
    rows = []
    with open(os.path.join(GOLDEN, "paper_restart_memory.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            meth, m, t, tol, *v = line.split()
            rows.append((meth, m, int(t), tol, *map(int, v)))
    return rows


def test_restart_cycle_memory_reproduces_paper_tables():
    # one restart at the flexible run's switch iteration sIt + 1; the block formed there
    # opens the second cycle; mem = the larger of the two cycles (Section 5.2 tables)
    rows = _restart_rows()
    assert len(rows) == 144
    for meth, m, t, tol, it_f, sit, mem_f, it_r, mem_r, it_rf, mem_rf in rows:
        assert ecg.memory_formula(t, it_f, sit) == mem_f, (meth, m, t, tol)
        same_t = ecg.EcgResult(x=None, it=it_r, switch_iters=[], widths=[t] * it_r, rho=[1.0], status="",
                               t_final=t, deflated=0, restart_iters=[sit + 1])
        assert same_t.mem_cycle == mem_r, (meth, m, t, tol)
        halved = ecg.EcgResult(x=None, it=it_rf, switch_iters=[sit + 1], rho=[1.0], status="",
                               widths=[t] * sit + [t // 2] * (it_rf - sit), t_final=t // 2, deflated=0,
                               restart_iters=[sit + 1])
        assert halved.mem_cycle == mem_rf, (meth, m, t, tol)


def test_restart_tol_fires_at_the_switch_iteration():
    # the restart test uses the switch statistic at the same point (Section 3), so a single
    # restart at restartTol happens where the flexible run with switchTol = restartTol halves
    p = W.config("poisson64")
    A = p.A.to_scipy()
    flex = ecg.flexible_sre_cg2(A, p.b, p.part, p.t, tol=p.tol, reduce=ecg.REDUCE_ONCE, switch_tol=1e-4)
    rs = ecg.flexible_sre_cg2(A, p.b, p.part, p.t, tol=p.tol, restart=ecg.RESTART_TOL, restart_tol=1e-4,
                              max_restarts=1)
    rf = ecg.flexible_sre_cg2(A, p.b, p.part, p.t, tol=p.tol, reduce=ecg.REDUCE_ONCE, switch_tol=1e-4,
                              restart_at_switch=True)
    assert rs.restart_iters == flex.switch_iters == rf.restart_iters == rf.switch_iters
    sit = flex.sit
    assert rs.mem_cycle == p.t * max(sit, rs.it - sit)
    assert rf.mem_cycle == max(p.t * sit, p.t // 2 * (rf.it - sit))
    assert rs.status == rf.status == "converged"
    # the iterates up to the restart are those of the unrestarted run
    assert rs.rho[:sit + 1] == flex.rho[:sit + 1]


@pytest.mark.parametrize("variant", ["sre", "msdo"])
def test_restarted_cycles_are_galerkin_projections_from_the_restart_point(variant):
    # restarting every j iterations: inside a cycle the iterate is the Galerkin projection
    # of the solution onto x_s + K_{i,t}(A, r_s) (SRE-CG2), or onto x_s + span{T(r_s), ...}
    # (MSDO-CG), with x_s the iterate at the restart (50-digit definitions)
    A, b, part = tiny(n=40, t=4, kappa=30.0, seed=53)
    j = 3
    if variant == "sre":
        res = ecg.flexible_sre_cg2(A, b, part, 4, tol=1e-14, kmax=9, restart=ecg.RESTART_EVERY,
                                   restart_every=j, record=True)
    else:
        res = ecg.flexible_msdo_cg(A, b, part, 4, tol=1e-14, kmax=9, restart=ecg.RESTART_EVERY,
                                   restart_every=j, record=True)
    assert res.restart_iters == [4, 7] and res.mem_cycle == 4 * j
    for start in (0, 3, 6):
        xs = np.zeros(len(b)) if start == 0 else res.iterates[start - 1]
        for i in range(1, j + 1):
            if start + i > res.it:
                break
            if variant == "sre":
                ref = brute.krylov_projection(A, b, part, 4, i, x0=xs)
            else:
                ref = brute.msdo_projection(A, b, part, 4, i, x0=xs)[-1]
            got = res.iterates[start + i - 1]
            assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref), (start, i)


def test_restart_beyond_the_run_changes_nothing():
    A, b, part = tiny(n=48, t=4, kappa=1e3, seed=57)
    ref = ecg.flexible_sre_cg2(A, b, part, 4, tol=1e-10)
    res = ecg.flexible_sre_cg2(A, b, part, 4, tol=1e-10, restart=ecg.RESTART_EVERY, restart_every=ref.it + 1)
    assert res.restart_iters == [] and res.it == ref.it and np.array_equal(res.x, ref.x)


def test_oracle_memory_matches_its_switch_bookkeeping():
    p = W.config("poisson64")
    A = p.A.to_scipy()
    res = ecg.flexible_sre_cg2(A, p.b, p.part, p.t, reduce=ecg.REDUCE_ONCE, switch_tol=1e-4, t_min=2)
    assert len(res.switch_iters) == 1 and res.deflated == 0
    assert res.mem == ecg.memory_formula(p.t, res.it, res.sit)


def test_switch_rule_uses_absolute_change():
    # tol1 = |rho_k - rho_{k-1}| / rho_0: the residual norm may rise, which must
    # not trigger a switch (without the absolute value every run would switch at k=2)
    A, b, part = tiny(n=48, t=8, kappa=1e3, seed=23)
    res = ecg.flexible_sre_cg2(A, b, part, 8, tol=1e-10, reduce=ecg.REDUCE_ONCE, switch_tol=1e-6, t_min=1)
    rho = np.array(res.rho)
    d = np.abs(np.diff(rho)) / rho[0]
    if res.switch_iters:
        k = res.switch_iters[0]
        assert d[k - 2] < 1e-6 and np.all(d[: k - 2] >= 1e-6)
    else:
        assert np.all(d[:-1] >= 1e-6)


def test_repeated_halving_reaches_t_min():
    p = W.config("jump3d160", scale=8)
    A = p.A.to_scipy()
    res = ecg.flexible_sre_cg2(A, p.b, p.part, p.t, reduce=ecg.REDUCE_REPEAT, switch_tol=1e-2, t_min=8,
                               kmax=400)
    widths = sorted(set(res.widths), reverse=True)
    assert widths[0] == 64 and widths[-1] >= 8
    assert all(w in (64, 32, 16, 8) for w in widths)
    assert res.t_final == widths[-1]


@pytest.mark.parametrize("t,kw", [(5, dict(reduce=ecg.REDUCE_ONCE)), (6, dict(reduce=ecg.REDUCE_REPEAT)),
                                  (12, dict(reduce=ecg.REDUCE_SCHEDULE, schedule=[2, 3, 4]))])
def test_halving_an_odd_width_is_rejected(t, kw):
    # subdomains merge in pairs (2i, 2i+1; Section 4): an odd width cannot be halved
    A, b, part = tiny(n=48, t=t, seed=5)
    with pytest.raises(ValueError):
        ecg.flexible_sre_cg2(A, b, part, t, t_min=1, **kw)
    with pytest.raises(ValueError):
        ecg.flexible_msdo_cg(A, b, part, t, t_min=1, **kw)
    # a t_min that stops the halving before the odd width is accepted
    ecg.flexible_sre_cg2(A, b, part, t, t_min=t // 2 if t % 2 == 0 else t, kmax=3, **kw)


# ---------------------------------------------------------------- deflation and failures
def test_zero_subdomain_residual_is_deflated():
    A, b, part = tiny(n=40, t=4, seed=29)
    b = b.copy()
    b[part == 2] = 0.0
    res = ecg.flexible_sre_cg2(A, b, part, 4, tol=1e-10)
    assert res.widths[0] == 3 and res.status == "converged"
    x = np.linalg.solve(A, b)
    assert np.linalg.norm(res.x - x) <= 1e-8 * np.linalg.norm(x)


def test_breakdown_without_deflation():
    A, b, part = tiny(n=40, t=4, seed=29)
    b = b.copy()
    b[part == 2] = 0.0
    res = ecg.flexible_sre_cg2(A, b, part, 4, tol=1e-10, deflate_tol=-1.0)
    assert res.status == "breakdown"


def test_noise_columns_deflated_past_exact_termination():
    # after n/t iterations the Krylov space is the whole space; the next candidate, once
    # A-orthonormalised against it, is rounding noise relative to its norm beforehand, so
    # every column is dropped (breakdown) and exactly n A-orthonormal vectors were stored
    for n, t in [(48, 4), (60, 6)]:
        A, b, part = tiny(n=n, t=t, seed=17)
        res = ecg.flexible_sre_cg2(A, b, part, t, tol=1e-30, kmax=n // t + 4, record=True)
        assert res.status == "breakdown" and res.it == n // t and res.mem == n
        x = np.linalg.solve(A, b)
        assert np.linalg.norm(res.x - x) <= 1e-10 * np.linalg.norm(x)


def test_kmax_gives_not_converged():
    # the loop guard is k < k_max (Algorithm 3), so at most k_max - 1 iterations
    A, b, part = tiny(n=48, t=4, kappa=1e3, seed=31)
    res = ecg.flexible_sre_cg2(A, b, part, 4, tol=1e-12, kmax=3)
    assert res.it == 2 and res.status == "not_converged"


# ---------------------------------------------------------------- preconditioning (Section 4.5)
def test_split_preconditioned_equals_run_on_transformed_system():
    # option 2 (modified recurrences on Z_k = L^{-T} Z-hat_k) reproduces option 1
    # (the method on A-hat = L^{-1} A L^{-T}, b-hat = L^{-1} b, x = L^{-T} x-hat)
    A, b, part = tiny(n=40, t=4, kappa=1e3, seed=37)
    rng = np.random.default_rng(5)
    L = np.tril(rng.uniform(-0.3, 0.3, (40, 40)), -1) + np.diag(rng.uniform(1.0, 2.0, 40))
    Linv = np.linalg.inv(L)
    Ah = Linv @ A @ Linv.T
    bh = Linv @ b
    hat = ecg.flexible_sre_cg2(Ah, bh, part, 4, tol=1e-30, kmax=6, record=True)
    pre = ecg.SplitPreconditioner(lambda X: Linv @ X, lambda X: Linv.T @ X)
    res = ecg.flexible_sre_cg2(A, b, part, 4, tol=1e-30, kmax=6, record=True, precond=pre)
    for k in range(5):
        xk = Linv.T @ hat.iterates[k]
        assert np.linalg.norm(res.iterates[k] - xk) <= 1e-10 * np.linalg.norm(xk)


# ---------------------------------------------------------------- IC(0) block Jacobi (Section 5.3)
def test_ic0_is_exact_cholesky_without_fill():
    # a tridiagonal SPD matrix has no fill-in, so IC(0) is its Cholesky factor (LAPACK)
    import scipy.sparse as sp

    from oracle import precond

    n = 30
    rng = np.random.default_rng(3)
    off = -rng.uniform(0.2, 1.0, n - 1)
    d = np.abs(np.r_[0, off]) + np.abs(np.r_[off, 0]) + rng.uniform(0.1, 1.0, n)
    A = sp.diags([off, d, off], [-1, 0, 1], format="csr")
    L = precond.ic0(A).toarray()
    assert np.allclose(L, np.linalg.cholesky(A.toarray()), rtol=0, atol=1e-13)


def test_ic0_matches_a_on_its_pattern():
    # defining property of IC(0): (L L^T)_ij = a_ij for every (i, j) in the pattern of A
    from oracle import precond

    p = W.config("learn2d256", seed=3, scale=8)
    A = p.A.to_scipy()
    Ab = precond.block_diagonal_part(A, p.part)
    L = precond.ic0(Ab)
    LLT = (L @ L.T).tocsr()
    coo = Ab.tocoo()
    assert np.abs(np.asarray(LLT[coo.row, coo.col]).ravel() - coo.data).max() <= 1e-12 * np.abs(coo.data).max()
    # couplings across subdomains are absent from L
    Lc = L.tocoo()
    assert np.all(p.part[Lc.row] == p.part[Lc.col])


def test_block_jacobi_commutes_with_split():
    # Section 4.5: for a block-diagonal M on the t subdomains, L^{-T} T(L^{-1} r) = M^{-1} T(r)
    from oracle import precond

    p = W.config("learn2d256", seed=4, scale=8)
    A = p.A.to_scipy()
    pre, _ = precond.bj_ic0_preconditioner(A, p.part)
    r = W.rhs_uniform(p.n, 9)
    lhs = pre.linvT(ecg.split(pre.linv(r), p.part, p.t))
    rhs = pre.minv(ecg.split(r, p.part, p.t))
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()
    # also after one halving (merged subdomains are unions of the original blocks)
    lhs = pre.linvT(ecg.split(pre.linv(r), p.part >> 1, p.t // 2))
    rhs = pre.minv(ecg.split(r, p.part >> 1, p.t // 2))
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


# ---------------------------------------------------------------- block-Jacobi Cholesky, 64 blocks (Section 5.3)
def _chol64(scale=8):
    p = W.config("jump2d512", scale=scale)  # 64x64 grid at scale 8
    blocks = W.box_partition(p.grid, (8, 8))  # 64 blocks; the 4x8 subdomains are pairs of them
    return p, blocks


def test_block_cholesky_reproduces_the_block_diagonal():
    from oracle import precond

    p, blocks = _chol64()
    assert np.array_equal(blocks >> 1, p.part)
    A = p.A.to_scipy()
    L = precond.block_cholesky(A, blocks)
    Ab = precond.block_diagonal_part(A, blocks)
    assert abs(L @ L.T - Ab).max() <= 1e-12 * abs(Ab).max()
    Lc = L.tocoo()
    assert np.all(blocks[Lc.row] == blocks[Lc.col]) and np.all(Lc.row >= Lc.col)
    assert L.diagonal().min() > 0
    # exact factor: fill inside the band, unlike IC(0)
    assert L.nnz > precond.ic0(Ab).nnz


def test_one_block_cholesky_solves_in_one_iteration():
    # M = A: the preconditioned operator is the identity and r_hat_0 is the sum of the
    # columns of T(r_hat_0), so the first Galerkin iterate is exact (SRE-CG2 and MSDO-CG)
    from oracle import precond

    p = W.config("learn2d256", seed=5, scale=8)
    A = p.A.to_scipy()
    pre, _ = precond.bj_chol_preconditioner(A, np.zeros(p.n, dtype=np.int32))
    xs = spl_solve(A, p.b)
    for fn in (ecg.flexible_sre_cg2, ecg.flexible_msdo_cg):
        res = fn(A, p.b, p.part, p.t, tol=1e-10, precond=pre)
        assert res.it == 1 and res.status == "converged"
        assert np.linalg.norm(res.x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_block_cholesky_commutes_with_split_on_unions_of_blocks():
    # the t subdomains are unions of the 64 blocks, so L is block diagonal on them too
    from oracle import precond

    p, blocks = _chol64()
    A = p.A.to_scipy()
    pre, _ = precond.bj_chol_preconditioner(A, blocks)
    r = W.rhs_uniform(p.n, 9)
    for lvl in (0, 1):
        part, t = p.part >> lvl, p.t >> lvl
        lhs = pre.linvT(ecg.split(pre.linv(r), part, t))
        rhs = pre.minv(ecg.split(r, part, t))
        assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


# ---------------------------------------------------------------- learned G G^T (oracle)
def _learn_case(seed=3, scale=16):
    from oracle import learned as Lr

    p = W.config("learn2d256", seed=seed, scale=scale)  # 16x16 grid
    A = p.A.to_scipy()
    nx = p.grid[0]
    a5 = Lr.stencil5(A, nx)
    x = np.linalg.solve(A.toarray(), p.b)
    return p, A, nx, a5, x


def test_learned_zero_output_is_jacobi_and_spd():
    from oracle import learned as Lr

    p, A, nx, a5, x = _learn_case()
    o = np.zeros((p.n, 3))
    G = Lr.g_matrix(*Lr.g_diagonals(o, a5, nx), nx).toarray()
    assert np.allclose(G @ G.T, np.diag(1.0 / A.diagonal()), rtol=1e-14, atol=0)
    theta = Lr.init_params(5)
    theta[-99:] = 0.05 * np.random.default_rng(1).standard_normal(99)  # non-zero last layer
    o, _ = Lr.mlp_forward(theta, Lr.features(a5, nx))
    G = Lr.g_matrix(*Lr.g_diagonals(o, a5, nx), nx).toarray()
    assert np.all(np.diag(G) > 0) and np.allclose(np.triu(G, 1), 0)
    assert np.linalg.eigvalsh(G @ G.T).min() > 0


def test_stencil5_reassembles_operator():
    from oracle import learned as Lr

    p, A, nx, a5, x = _learn_case(seed=4)
    n = p.n
    v = np.random.default_rng(2).standard_normal(n)
    y = a5[0] * v
    y[1:] += a5[1][1:] * v[:-1]
    y[:-1] += a5[2][:-1] * v[1:]
    y[nx:] += a5[3][nx:] * v[:-nx]
    y[:-nx] += a5[4][:-nx] * v[nx:]
    assert np.allclose(y, A @ v, rtol=1e-14, atol=1e-12 * np.abs(A @ v).max())


def test_learned_gradient_matches_finite_differences():
    # central differences of the batch loss in random parameter directions (FP64)
    from oracle import learned as Lr

    p, A, nx, a5, x = _learn_case(seed=6)
    rng = np.random.default_rng(7)
    theta = Lr.init_params(8)
    theta += 0.05 * rng.standard_normal(theta.shape)
    ops = [(A, a5, p.b, x)]
    L0, g = Lr.batch_loss_and_grad(theta, ops, nx)
    for _ in range(4):
        d = rng.standard_normal(theta.shape)
        h = 1e-5
        Lp, _ = Lr.batch_loss_and_grad(theta + h * d, ops, nx)
        Lm, _ = Lr.batch_loss_and_grad(theta - h * d, ops, nx)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * max(abs(fd), 1e-3)


def test_learned_g_gradient_matches_finite_differences():
    # the closed-form dL/dG_ij = (2/c)((Ae)_i u_j + b_i w_j) against differences of L
    from oracle import learned as Lr

    p, A, nx, a5, x = _learn_case(seed=9)
    rng = np.random.default_rng(3)
    o = 0.1 * rng.standard_normal((p.n, 3))
    gd, gw, gs = Lr.g_diagonals(o, a5, nx)
    L, (dgd, dgw, dgs) = Lr.loss_and_grad_g(A, Lr.g_matrix(gd, gw, gs, nx), p.b, x, nx)
    for arr, darr in ((gd, dgd), (gw, dgw), (gs, dgs)):
        for j in rng.choice(np.nonzero(arr)[0], 5, replace=False):
            h = 1e-6 * max(abs(arr[j]), 1e-3)
            arr[j] += h
            Lp, _ = Lr.loss_and_grad_g(A, Lr.g_matrix(gd, gw, gs, nx), p.b, x, nx)
            arr[j] -= 2 * h
            Lm, _ = Lr.loss_and_grad_g(A, Lr.g_matrix(gd, gw, gs, nx), p.b, x, nx)
            arr[j] += h
            assert abs((Lp - Lm) / (2 * h) - darr[j]) <= 1e-5 * max(abs(darr[j]), 1e-8) + 1e-9


def test_adam_first_step_is_signed_learning_rate():
    # with bias correction the first Adam step moves every coordinate by lr * g/(|g|+eps)
    from oracle import learned as Lr

    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th, m, v = Lr.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


# ---------------------------------------------------------------- MSDO-CG (Section 2.2, Algorithms 2 and 4)
def test_msdo_iterates_equal_modified_subspace_projection():
    # both MSDO-CG and modified MSDO-CG are the Galerkin iterates on span{T(r_0),...,T(r_{k-1})}
    A, b, part = tiny(n=40, t=4, kappa=30.0, seed=41)
    xs = brute.msdo_projection(A, b, part, 4, 6)
    ms = ecg.flexible_msdo_cg(A, b, part, 4, tol=1e-14, kmax=7, record=True)
    mm = ecg.flexible_sre_cg2(A, b, part, 4, tol=1e-14, kmax=7, record=True, candidate="modified-msdo")
    for k in range(6):
        assert np.linalg.norm(ms.iterates[k] - xs[k]) <= 1e-11 * np.linalg.norm(xs[k])
        assert np.linalg.norm(mm.iterates[k] - xs[k]) <= 1e-11 * np.linalg.norm(xs[k])


def test_flexible_msdo_iterates_with_switch():
    A, b, part = tiny(n=40, t=8, kappa=30.0, seed=43)
    xs = brute.msdo_projection(A, b, part, 8, 6, [3])
    ms = ecg.flexible_msdo_cg(A, b, part, 8, tol=1e-14, kmax=7, record=True, reduce=ecg.REDUCE_SCHEDULE,
                              schedule=[3])
    # a column can be dependent (a subdomain with a single unknown gives parallel splits)
    assert ms.switch_iters == [3] and ms.widths[0] == 8 and max(ms.widths[2:6]) <= 4
    for k in range(6):
        assert np.linalg.norm(ms.iterates[k] - xs[k]) <= 1e-11 * np.linalg.norm(xs[k])


def test_msdo_a_orthonormal_and_memory():
    p = W.config("poisson64")
    A = p.A.to_scipy()
    r = ecg.flexible_msdo_cg(A, p.b, p.part, p.t, tol=1e-8, reduce=ecg.REDUCE_ONCE, switch_tol=1e-4, t_min=2,
                             record=True)
    assert r.status == "converged" and len(r.switch_iters) == 1
    assert r.mem == ecg.memory_formula(p.t, r.it, r.sit)
    Q = np.hstack([B[:, np.any(B != 0, axis=0)] for B in r.blocks[:20]])
    assert np.abs(Q.T @ (A @ Q) - np.eye(Q.shape[1])).max() <= 1e-10
