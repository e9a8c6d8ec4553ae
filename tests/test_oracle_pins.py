"""More pins of the FP64 oracle: the factorised preconditioner, the learned part's features,
network and optimiser, classical CG, and MSDO-CG's beta term.

Each expected value is either worked out by hand (written here as literals, with the
arithmetic in the comments) or comes from an independent definition: the method run on the
explicitly transformed system, a 50-digit Galerkin projection, or a property the
mathematics fixes.
"""

import math

import mpmath as mp
import numpy as np
import scipy.sparse as sp

import workloads as W
from oracle import brute, ecg
from oracle import learned as Lr
from oracle import precond as opc


def _tiny(n=40, t=4, kappa=50.0, seed=1):
    A = W.random_spd(n, kappa, seed)
    b = W.rhs_uniform(n, seed + 1)
    part = W.random_partition(n, t, seed + 2)
    return A, b, part


def _lower_factor(n, seed):
    rng = np.random.default_rng(seed)
    return np.tril(rng.uniform(-0.4, 0.4, (n, n)), -1) + np.diag(rng.uniform(0.5, 2.0, n))


# ---------------------------------------------------------------- M^{-1} = G G^T (Section 4.5)
def test_factor_preconditioner_is_the_run_on_g_transpose_a_g():
    # Section 4.5: with M^{-1} = G G^T the split factors are L^{-1} = G^T and L^{-T} = G, so
    # option 2 (eq. (zsre2)) must reproduce the method run on A-hat = G^T A G, b-hat = G^T b,
    # mapped back by x = G x-hat.  G is dense and far from symmetric, so taking G G^T as
    # G^T G (or L^{-1} = G) gives a different A-hat and fails here.
    A, b, part = _tiny(n=40, t=4, kappa=200.0, seed=51)
    G = _lower_factor(40, 52)
    assert np.linalg.norm(G @ G.T - G.T @ G) > 0.5 * np.linalg.norm(G @ G.T)
    Ah = G.T @ A @ G
    bh = G.T @ b
    hat = ecg.flexible_sre_cg2(Ah, bh, part, 4, tol=1e-30, kmax=7, record=True, reduce=ecg.REDUCE_SCHEDULE,
                               schedule=[4])
    pre = opc.factor_preconditioner(sp.csr_matrix(G))
    res = ecg.flexible_sre_cg2(A, b, part, 4, tol=1e-30, kmax=7, record=True, precond=pre,
                               reduce=ecg.REDUCE_SCHEDULE, schedule=[4])
    assert res.switch_iters == hat.switch_iters == [4]
    for k in range(6):
        xk = G @ hat.iterates[k]
        assert np.linalg.norm(res.iterates[k] - xk) <= 1e-10 * np.linalg.norm(xk)
    # and the preconditioned residual history is the transformed one: r = A x - b, r-hat = G^T r
    for k in range(6):
        rk = b - A @ res.iterates[k]
        assert np.linalg.norm(G.T @ rk - hat.residuals[k]) <= 1e-9 * np.linalg.norm(bh)


def test_factor_preconditioner_msdo_is_the_run_on_g_transpose_a_g():
    # the same equivalence for split-preconditioned MSDO-CG (Algorithm 5)
    A, b, part = _tiny(n=36, t=4, kappa=100.0, seed=53)
    G = _lower_factor(36, 54)
    hat = ecg.flexible_msdo_cg(G.T @ A @ G, G.T @ b, part, 4, tol=1e-30, kmax=6, record=True)
    res = ecg.flexible_msdo_cg(A, b, part, 4, tol=1e-30, kmax=6, record=True,
                               precond=opc.factor_preconditioner(sp.csr_matrix(G)))
    for k in range(5):
        xk = G @ hat.iterates[k]
        assert np.linalg.norm(res.iterates[k] - xk) <= 1e-10 * np.linalg.norm(xk)


# ---------------------------------------------------------------- learned part: features, network, Adam
def _hand_operator_3x3():
    """5-point operator on a 3 x 3 grid (x fastest): diagonal 4..12, west-east couplings of
    the pairs (0,1) (1,2) (3,4) (4,5) (6,7) (7,8) = -1 -2 -3 -0.5 -1.5 -2.5, south-north
    couplings of (0,3) (1,4) (2,5) (3,6) (4,7) (5,8) = -0.25 -0.75 -1.25 -1.75 -2.25 -0.125."""
    A = np.diag(np.arange(4.0, 13.0))
    for (i, j), v in zip([(0, 1), (1, 2), (3, 4), (4, 5), (6, 7), (7, 8)], [-1, -2, -3, -0.5, -1.5, -2.5]):
        A[i, j] = A[j, i] = v
    for (i, j), v in zip([(0, 3), (1, 4), (2, 5), (3, 6), (4, 7), (5, 8)], [-0.25, -0.75, -1.25, -1.75, -2.25, -0.125]):
        A[i, j] = A[j, i] = v
    return A


def test_features_of_a_hand_worked_3x3_stencil():
    A = _hand_operator_3x3()
    a5 = Lr.stencil5(sp.csr_matrix(A), 3)
    F = Lr.features(a5, 3)
    # f = (log a_ii, a_iW/a_ii, a_iE/a_ii, a_iS/a_ii, a_iN/a_ii, log(a_WW/a_ii), log(a_SS/a_ii))
    want = {
        # corner (0,0): east a_01 = -1, north a_03 = -0.25, no west or south neighbour
        0: [math.log(4.0), 0.0, -0.25, 0.0, -0.0625, 0.0, 0.0],
        # centre (1,1): a_44 = 8, west a_43 = -3, east a_45 = -0.5, south a_41 = -0.75,
        # north a_47 = -2.25, a_33 = 7, a_11 = 5
        4: [math.log(8.0), -0.375, -0.0625, -0.09375, -0.28125, math.log(0.875), math.log(0.625)],
        # (2,1): a_55 = 9, west a_54 = -0.5, south a_52 = -1.25, north a_58 = -0.125, a_44 = 8, a_22 = 6
        5: [math.log(9.0), -0.5 / 9, 0.0, -1.25 / 9, -0.125 / 9, math.log(8.0 / 9), math.log(6.0 / 9)],
        # (2,2): a_88 = 12, west a_87 = -2.5, south a_85 = -0.125, a_77 = 11, a_55 = 9
        8: [math.log(12.0), -2.5 / 12, 0.0, -0.125 / 12, 0.0, math.log(11.0 / 12), math.log(0.75)],
    }
    for i, f in want.items():
        assert np.allclose(F[i], f, rtol=1e-15, atol=1e-16), (i, F[i], f)


def _hand_params():
    """W1[0,0] = 1, W1[1,1] = 2, b1[1] = ln 2, W2[0,0] = 1, W2[0,1] = -1, W2[2,1] = 0.5,
    b2[2] = 0.25, W3[0,0] = 1, W3[1,2] = 2, W3[2,0] = -1, b3 = (0.1, 0.2, 0.3); all else 0.
    Flat offsets: W1 0, b1 224, W2 256, b2 1280, W3 1312, b3 1408 (row-major matrices)."""
    th = np.zeros(Lr.NPARAM)
    th[0] = 1.0
    th[1 * 7 + 1] = 2.0
    th[224 + 1] = math.log(2.0)
    th[256 + 0] = 1.0
    th[256 + 1] = -1.0
    th[256 + 2 * 32 + 1] = 0.5
    th[1280 + 2] = 0.25
    th[1312 + 0] = 1.0
    th[1312 + 32 + 2] = 2.0
    th[1312 + 64 + 0] = -1.0
    th[1408:1411] = [0.1, 0.2, 0.3]
    return th


def test_mlp_forward_and_output_map_by_hand():
    A = _hand_operator_3x3()
    a5 = Lr.stencil5(sp.csr_matrix(A), 3)
    F = Lr.features(a5, 3)
    o, _ = Lr.mlp_forward(_hand_params(), F)
    # row 0: f_0 = ln 4, f_1 = 0.  h1_0 = tanh(ln 4) = 15/17, h1_1 = tanh(ln 2) = 3/5;
    # h2_0 = tanh(15/17 - 3/5) = tanh(24/85), h2_2 = tanh(0.5 * 3/5 + 0.25) = tanh(0.55), h2_1 = 0;
    # o = (h2_0 + 0.1, 2 h2_2 + 0.2, -h2_0 + 0.3)
    h20, h22 = math.tanh(24.0 / 85.0), math.tanh(0.55)
    assert np.allclose(o[0], [h20 + 0.1, 2 * h22 + 0.2, -h20 + 0.3], rtol=1e-14, atol=0)
    # row 4: f_0 = ln 8, f_1 = -0.375.  h1_0 = tanh(ln 8) = 63/65, h1_1 = tanh(ln 2 - 0.75)
    h10, h11 = 63.0 / 65.0, math.tanh(math.log(2.0) - 0.75)
    h20, h22 = math.tanh(h10 - h11), math.tanh(0.5 * h11 + 0.25)
    assert np.allclose(o[4], [h20 + 0.1, 2 * h22 + 0.2, -h20 + 0.3], rtol=1e-14, atol=0)
    # output map: G_ii = a_ii^{-1/2} exp(o_0), G_i,i-1 = a_ii^{-1/2} o_1 (0 on the west
    # boundary), G_i,i-nx = a_ii^{-1/2} o_2 (0 on the south boundary)
    gd, gw, gs = Lr.g_diagonals(o, a5, 3)
    assert math.isclose(gd[4], math.exp(o[4, 0]) / math.sqrt(8.0), rel_tol=1e-15)
    assert math.isclose(gw[4], o[4, 1] / math.sqrt(8.0), rel_tol=1e-15)
    assert math.isclose(gs[4], o[4, 2] / math.sqrt(8.0), rel_tol=1e-15)
    assert gw[0] == 0.0 and gs[0] == 0.0 and gw[3] == 0.0 and gs[2] == 0.0 and gw[1] != 0.0 and gs[3] != 0.0
    G = Lr.g_matrix(gd, gw, gs, 3).toarray()
    assert G[4, 3] == gw[4] and G[4, 1] == gs[4] and G[4, 4] == gd[4] and np.allclose(np.triu(G, 1), 0)


def test_adam_three_steps_by_hand():
    # Kingma and Ba with beta1 = 1/2, beta2 = 3/4, lr = 1, eps = 0, gradients 1, -2, 3 from 0:
    # step 1: m = 1/2, v = 1/4; m-hat = 1, v-hat = 1; theta = -1
    # step 2: m = 1/4 - 1 = -3/4, v = 3/16 + 1 = 19/16; m-hat = (-3/4)/(3/4) = -1,
    #         v-hat = (19/16)/(7/16) = 19/7; theta = -1 + sqrt(7/19)
    # step 3: m = -3/8 + 3/2 = 9/8, v = 57/64 + 9/4 = 201/64; m-hat = (9/8)/(7/8) = 9/7,
    #         v-hat = (201/64)/(37/64) = 201/37; theta = -1 + sqrt(7/19) - (9/7) sqrt(37/201)
    th, m, v = np.zeros(1), np.zeros(1), np.zeros(1)
    want = [(-1.0, 0.5, 0.25), (-1.0 + math.sqrt(7 / 19), -0.75, 19 / 16),
            (-1.0 + math.sqrt(7 / 19) - (9 / 7) * math.sqrt(37 / 201), 9 / 8, 201 / 64)]
    for step, (g, (wt, wm, wv)) in enumerate(zip([1.0, -2.0, 3.0], want), start=1):
        th, m, v = Lr.adam_step(th, np.array([g]), m, v, step, lr=1.0, beta1=0.5, beta2=0.75, eps=0.0)
        assert math.isclose(th[0], wt, rel_tol=1e-15) and math.isclose(m[0], wm, rel_tol=1e-15)
        assert math.isclose(v[0], wv, rel_tol=1e-15)


def test_adam_constant_gradient_moves_lr_per_step():
    # with a constant gradient g the bias-corrected moments are exactly g and g^2 at every
    # step, so each step moves by lr * g / (|g| + eps), at step 1 and at step 50 alike
    g = np.array([0.7, -3.0, 2e-3])
    th, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for step in range(1, 51):
        prev = th
        th, m, v = Lr.adam_step(th, g, m, v, step, lr=0.01)
        assert np.allclose(th - prev, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=0), step


# ---------------------------------------------------------------- classical CG (Section 1)
def test_cg_iterates_are_krylov_galerkin_projections():
    # CG's k-th iterate is the Galerkin projection on x0 + K_k(A, r0): the t = 1 case of the
    # enlarged subspace, evaluated in 50 digits with a monomial basis
    A, b, _ = _tiny(n=30, t=1, kappa=40.0, seed=61)
    x0 = W.rhs_uniform(30, 62)
    _, k, its = ecg.cg(A, b, x0=x0, tol=1e-30, kmax=8, record=True)
    assert k == 8
    for j in (1, 3, 5, 8):
        xk = brute.krylov_projection(A, b, np.zeros(30, dtype=np.int64), 1, j, x0=x0)
        assert np.linalg.norm(its[j - 1] - xk) <= 1e-11 * np.linalg.norm(xk), j


def test_cg_solves_and_stops_on_relative_residual():
    A, b, _ = _tiny(n=40, t=1, kappa=100.0, seed=63)
    x, k, _ = ecg.cg(A, b, tol=1e-10)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    _, k1, _ = ecg.cg(A, b, tol=1e-10, kmax=k - 1)
    assert k1 == k - 1  # k_max bounds the iterations


# ---------------------------------------------------------------- MSDO-CG's beta (eq. (pk), Algorithm 2)
def test_msdo_candidate_sum_is_a_orthogonal_to_previous_block():
    # P_k = [T(r_{k-1})] + P_{k-1} diag(beta_k), beta_k = -V_{k-1}^T r_{k-1}, V = A P.  Its
    # columns sum to r_{k-1} + P_{k-1} beta_k = (I - P_{k-1} P_{k-1}^T A) r_{k-1}, which is
    # A-orthogonal to the A-orthonormal P_{k-1}.  A sign error or a transposition in beta breaks
    # it (CGS2 against Q hides beta from the iterates, which is why this is checked here).
    A, b, part = _tiny(n=40, t=4, kappa=60.0, seed=71)
    r = ecg.flexible_msdo_cg(A, b, part, 4, tol=1e-14, kmax=8, record=True)
    for k in range(2, 8):
        P_prev, cand = r.blocks[k - 2], r.candidates[k - 1]
        s = cand.sum(axis=1)
        assert np.abs(P_prev.T @ (A @ s)).max() <= 1e-12 * np.linalg.norm(A @ s) * np.abs(P_prev).max() * 40
        # and beta is not trivially zero
        assert np.linalg.norm(cand - ecg.split(b - A @ r.iterates[k - 2], part, 4)) > 1e-3 * np.linalg.norm(cand)


def test_msdo_preconditioned_candidate_sum_is_a_orthogonal_to_previous_block():
    # Algorithm 5: beta_k = -V_{k-1}^T M^{-1} r_{k-1} and the split term L^{-T}[T(L^{-1} r)];
    # the columns sum to M^{-1} r_{k-1} + P_{k-1} beta_k, again A-orthogonal to P_{k-1}
    A, b, part = _tiny(n=40, t=4, kappa=60.0, seed=73)
    G = _lower_factor(40, 74)
    r = ecg.flexible_msdo_cg(A, b, part, 4, tol=1e-14, kmax=7, record=True,
                             precond=opc.factor_preconditioner(sp.csr_matrix(G)))
    for k in range(2, 7):
        P_prev, s = r.blocks[k - 2], r.candidates[k - 1].sum(axis=1)
        assert np.abs(P_prev.T @ (A @ s)).max() <= 1e-11 * np.linalg.norm(A @ s) * np.abs(P_prev).max() * 40


def test_msdo_second_candidate_in_50_digits():
    # k = 2 of Algorithm 2 on two subdomains, worked in 50 digits: P_1 = A-orthonormal basis
    # of [T(r_0)] (positive diagonal, unique), V_1 = A P_1, alpha = P_1^T r_0,
    # r_1 = r_0 - V_1 alpha, beta = -V_1^T r_1, P_2 = [T(r_1)] + P_1 diag(beta)
    n = 12
    A, b, part = _tiny(n=n, t=2, kappa=20.0, seed=75)
    r = ecg.flexible_msdo_cg(A, b, part, 2, tol=1e-14, kmax=3, record=True)
    with mp.workdps(50):
        Am = mp.matrix(A.tolist())
        r0 = mp.matrix([[mp.mpf(float(v))] for v in b])
        T0 = mp.matrix(n, 2)
        for i in range(n):
            T0[i, int(part[i])] = r0[i, 0]
        cols = []
        for j in range(2):
            v = T0[:, j]
            for q in cols:
                v = v - q * (q.T * Am * v)[0, 0]
            cols.append(v / mp.sqrt((v.T * Am * v)[0, 0]))
        P1 = mp.matrix(n, 2)
        for j in range(2):
            for i in range(n):
                P1[i, j] = cols[j][i, 0]
        V1 = Am * P1
        r1 = r0 - V1 * (P1.T * r0)
        beta = -(V1.T * r1)
        P2 = mp.matrix(n, 2)
        for i in range(n):
            P2[i, int(part[i])] = r1[i, 0]
            for j in range(2):
                P2[i, j] += P1[i, j] * beta[j, 0]
        want = np.array([[float(P2[i, j]) for j in range(2)] for i in range(n)])
    assert np.abs(r.candidates[1] - want).max() <= 1e-13 * np.abs(want).max()
