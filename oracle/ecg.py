"""FP64 oracle of flexibly enlarged CG (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It is deliberately plain: NumPy/SciPy
products, LAPACK QR and Cholesky, no blocking or fusion.

What it follows
---------------
* The enlarged Krylov subspace and the split operator T^t (Section 1 and
  Section 2; the matrix [T^t(v)] of eq. (Tt) in Section 4): column j of
  [T^t(v)] holds the entries of v on subdomain delta_j and zeros elsewhere.
* SRE-CG2 (Section 2.1, Algorithm 1) and its flexible form (Section 4.3,
  Algorithm 3): W_1 = [T^t(r_0)]; W_k = A W_{k-1}, or [T^{t/2}(r_{k-1})] at a
  switch; W_k is A-orthonormalised against all stored blocks Q (or the last
  ``trunc`` blocks, Section 3) and then against itself; alpha_k = W_k^T r_{k-1},
  x_k = x_{k-1} + W_k alpha_k, r_k = r_{k-1} - A W_k alpha_k.
* The switch test (Section 4.2): tol1 = |rho_k - rho_{k-1}| / rho_0, tested at
  the start of the next iteration; the halved partition merges subdomains 2i
  and 2i+1 (Section 4, definition of delta-tilde), i.e. ``part >> level``.
* Split preconditioning, option 2 (Section 4.5, eq. (zsre2)): the recurrences
  are unchanged and only the candidate block changes:
  L^{-T}[T(L^{-1} r)] at k = 1 and at a switch, M^{-1} A W_{k-1} otherwise.
* A-orthonormalisation (Section 5 names CGS2 and Pre-CholQR): against Q,
  two classical Gram-Schmidt passes in the A inner product,
  W <- W - Q (Q^T A W); then Pre-CholQR: a Euclidean thin QR W = W_hat R with
  positive diagonal, followed by S = W_hat^T A W_hat = C^T C (Cholesky) and
  W <- W_hat C^{-1}.

Readings where the paper is silent (stated again in the design notes):
* the absolute value in tol1 (the algorithms omit it, the text has it);
* rank deficiency: a column is dropped (deflated) when its Schur-complement pivot is
  <= deflate_tol times a reference: in the Euclidean QR step the column's squared norm
  before it was A-orthonormalised against the stored blocks, in the A step its own
  diagonal entry; a block whose columns are all dropped ends the solve (status
  "breakdown");
* repeated halving (rule REPEAT) and forced switch iterations (SCHEDULE)
  generalise the paper's single switch.
* restarts (Section 3): a restart at iteration k empties Q and takes the candidate
  [T(r_{k-1})] at the current width, as at k = 1.  RESTART_EVERY restarts when
  k mod j == 1; RESTART_TOL restarts when |rho_k - rho_{k-1}| / rho_c < restartTol,
  tested where the switch is tested, with rho_c the residual norm the current cycle
  started from (rho_0 before the first restart: a restarted cycle is a fresh solve from
  its own initial guess, while the stopping test keeps rho_0), at most max_restarts
  times (0 = no limit);
  restart_at_switch empties Q at every halving as well (the restarted flexible
  variants of the memory tables of Section 5.2).  A halving takes precedence over a
  restart in the same iteration.

Bookkeeping: ``it`` = completed iterations, ``switch_iters`` = iterations at
which a halved block was formed, ``mem`` = total stored columns (for one
switch this equals t*sIt + (t/2)*(It - sIt) with sIt = switch_iter - 1),
``restart_iters`` = iterations at which Q was emptied, ``mem_cycle`` = the largest
number of columns stored within one restart cycle (the mem of the restarted runs in
the Section 5.2 tables; equal to ``mem`` without restarts).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

REDUCE_NONE = 0
REDUCE_ONCE = 1
REDUCE_REPEAT = 2
REDUCE_SCHEDULE = 3

RESTART_NONE = 0
RESTART_EVERY = 1
RESTART_TOL = 2


def split(v: np.ndarray, part: np.ndarray, t: int) -> np.ndarray:
    """[T^t(v)]: n x t matrix, column j = v restricted to subdomain j (eq. (Tt))."""
    n = v.shape[0]
    out = np.zeros((n, t))
    out[np.arange(n), part] = v
    return out


def merged_partition(part: np.ndarray, level: int) -> np.ndarray:
    """Subdomain map after ``level`` halvings: delta-tilde_i = delta_{2i} U delta_{2i+1}."""
    return np.asarray(part) >> level


def _cholesky_pivot(S: np.ndarray) -> float:
    """Last pivot of the Cholesky factorisation of S (the Schur complement of the
    last diagonal entry), or -inf when the leading block is not positive definite."""
    try:
        c = np.linalg.cholesky(S)
    except np.linalg.LinAlgError:
        return -np.inf
    return float(c[-1, -1] ** 2)


def _select_columns(gram: np.ndarray, tau: float):
    """Greedy left-to-right column selection on a Gram matrix.

    Column j is kept when the Cholesky pivot of gram restricted to the kept
    columns plus j exceeds tau * gram[j, j].  tau < 0 keeps every column and
    reports failure instead (returns None) when a pivot is not positive.
    """
    m = gram.shape[0]
    d = np.diag(gram)
    try:  # common case: every column passes, one factorisation gives all pivots
        piv = np.diag(np.linalg.cholesky(gram)) ** 2
        if np.all(d > 0) and np.all(piv > (tau if tau > 0 else 0.0) * d):
            return list(range(m))
    except np.linalg.LinAlgError:
        pass
    keep = []
    for j in range(m):
        idx = keep + [j]
        p = _cholesky_pivot(gram[np.ix_(idx, idx)]) if d[j] > 0 else -np.inf
        if tau < 0:
            if not p > 0:
                return None
            keep.append(j)
        elif p > tau * d[j] and d[j] > 0:
            keep.append(j)
    return keep


def euclidean_qr(W: np.ndarray, tau: float, ref2=None):
    """Thin Householder QR with positive diagonal, dropping dependent columns.

    Column j is dropped when its distance to the span of the previously kept
    columns, squared, is <= tau * ref2[j] (ref2 defaults to ||w_j||^2; the solver passes
    the squared norms of the candidate before it was A-orthonormalised against the stored
    blocks, so a column that lay in their span is dropped even though what is left of it
    is rounding noise of its own size).  Returns (W_hat, kept indices), or
    (None, None) when tau < 0 and W is numerically rank deficient.
    """
    nrm2 = np.einsum("ij,ij->j", W, W) if ref2 is None else np.asarray(ref2, dtype=np.float64)
    m = W.shape[1]
    Qh, R = np.linalg.qr(W)
    d2 = np.diag(R) ** 2
    if np.all(nrm2 > 0) and np.all(d2 > (tau if tau > 0 else 0.0) * nrm2):
        keep = list(range(m))  # every prefix pivot passes: nothing to drop
    else:
        keep = []
        for j in range(m):
            if not nrm2[j] > 0:
                if tau < 0:
                    return None, None
                continue
            _, Rj = np.linalg.qr(W[:, keep + [j]])
            dj = Rj[-1, -1] ** 2
            if tau < 0:
                if not dj > 0:
                    return None, None
                keep.append(j)
            elif dj > tau * nrm2[j]:
                keep.append(j)
        if not keep:
            return np.zeros((W.shape[0], 0)), keep
        Qh, R = np.linalg.qr(W[:, keep])
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Qh * s[None, :], keep


def a_orthonormalize_self(W: np.ndarray, A, tau: float, keep_width: bool = False, ref2=None):
    """Pre-CholQR in the A inner product with deflation.

    Returns the A-orthonormal block (n x t_eff) or None on breakdown (tau < 0).  With
    keep_width the block keeps its t columns and a dropped column is a zero column in the
    position of the candidate column it came from (MSDO-CG pairs column j with subdomain j).
    """
    n, t = W.shape
    What, keep = euclidean_qr(W, tau, ref2)
    if What is None:
        return None
    if What.shape[1] == 0:
        return np.zeros((n, t)) if keep_width else What
    S = What.T @ (A @ What)
    S = 0.5 * (S + S.T)
    keep2 = _select_columns(S, tau)
    if keep2 is None:
        return None
    if not keep2:
        return np.zeros((n, t)) if keep_width else np.zeros((n, 0))
    S2 = S[np.ix_(keep2, keep2)]
    C = np.linalg.cholesky(S2).T  # upper, S2 = C^T C
    # W = W_hat C^{-1}  <=>  C^T W^T = W_hat^T
    Wn = sla.solve_triangular(C, What[:, keep2].T, trans="T", lower=False).T
    if not keep_width:
        return Wn
    full = np.zeros((n, t))
    full[:, [keep[j] for j in keep2]] = Wn
    return full


def a_orthonormalize_against(W: np.ndarray, Qm: np.ndarray, A) -> np.ndarray:
    """CGS2 in the A inner product: two passes of W <- W - Q (Q^T A W)."""
    for _ in range(2):
        W = W - Qm @ (Qm.T @ (A @ W))
    return W


class SplitPreconditioner:
    """M = L L^T given by two block operators: linv(X) = L^{-1} X, linvT(X) = L^{-T} X."""

    def __init__(self, linv, linvT):
        self.linv = linv
        self.linvT = linvT

    def minv(self, X):
        return self.linvT(self.linv(X))


@dataclass
class EcgResult:
    x: np.ndarray
    it: int
    switch_iters: list
    widths: list
    rho: list
    status: str
    t_final: int
    deflated: int
    iterates: list = field(default_factory=list)
    blocks: list = field(default_factory=list)
    residuals: list = field(default_factory=list)
    restart_iters: list = field(default_factory=list)
    candidates: list = field(default_factory=list)  # MSDO-CG: P_k before its A-orthonormalisation

    @property
    def mem(self) -> int:
        return int(sum(self.widths))

    @property
    def mem_cycle(self) -> int:
        """Largest sum of widths over the iterations of one restart cycle (a cycle starts
        at iteration 1 and at every restart iteration)."""
        best = cur = 0
        starts = set(self.restart_iters)
        for k, w in enumerate(self.widths, start=1):
            if k in starts:
                cur = 0
            cur += w
            best = max(best, cur)
        return int(best)

    @property
    def sit(self) -> int:
        """Iterations run at the initial width (the paper's sIt)."""
        return (self.switch_iters[0] - 1) if self.switch_iters else self.it

    @property
    def relres(self) -> float:
        return self.rho[-1] / self.rho[0] if self.rho[0] > 0 else 0.0


def _switch_now(rule, k, tol1, switch_tol, t_cur, t_min, switches, min_gap, schedule):
    if t_cur % 2 or t_cur // 2 < max(t_min, 1):
        return False
    if rule == REDUCE_NONE:
        return False
    if rule == REDUCE_SCHEDULE:
        return k in schedule
    if not tol1 < switch_tol:
        return False
    if rule == REDUCE_ONCE:
        return not switches
    if rule == REDUCE_REPEAT:
        return (not switches) or (k - switches[-1] >= min_gap)
    raise ValueError(rule)


def _check_halving(t, rule, t_min, schedule):
    """A halving merges subdomains 2i and 2i+1 (Section 4), so each width the rule may halve
    (down to t_min) must be even; raises ValueError otherwise."""
    steps = {REDUCE_NONE: 0, REDUCE_ONCE: 1, REDUCE_REPEAT: 64, REDUCE_SCHEDULE: len(schedule)}[rule]
    w = t
    for _ in range(steps):
        if w // 2 < max(t_min, 1):
            break
        if w % 2:
            raise ValueError(f"halving requested at odd block width {w}")
        w //= 2


def _restart_now(rule, k, tol1, every, restart_tol, restarts, max_restarts):
    if rule == RESTART_NONE:
        return False
    if rule == RESTART_EVERY:
        return (k - 1) % every == 0  # k mod j == 1 (Section 3)
    if rule == RESTART_TOL:
        return tol1 < restart_tol and (max_restarts <= 0 or len(restarts) < max_restarts)
    raise ValueError(rule)


def flexible_sre_cg2(A, b, part, t, *, x0=None, tol=1e-8, kmax=20000, reduce=REDUCE_NONE,
                     switch_tol=1e-5, t_min=1, min_gap=1, schedule=(), trunc=0,
                     deflate_tol=1e-14, precond: SplitPreconditioner | None = None,
                     record=False, candidate="sre", restart=RESTART_NONE, restart_every=0,
                     restart_tol=1e-5, max_restarts=0, restart_at_switch=False) -> EcgResult:
    """Flexibly SRE-CG2 (Algorithm 3); with reduce=REDUCE_NONE it is SRE-CG2
    (Algorithm 1), with trunc>0 the truncated SRE-CG2 of Section 3.

    A: anything with ``A @ X`` (dense array or scipy sparse), SPD, n x n.
    part: int array, subdomain of each unknown, values in [0, t).
    candidate: "sre" (W_k = A W_{k-1}) or "modified-msdo" (W_k = [T^t(r_{k-1})],
      the modified MSDO-CG of Section 2.2).
    restart, restart_every, restart_tol, max_restarts, restart_at_switch: the restarted
      variants of Section 3 (see the module notes).
    """
    b = np.asarray(b, dtype=np.float64)
    part = np.asarray(part)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    rho0 = float(np.linalg.norm(r))
    res = EcgResult(x=x, it=0, switch_iters=[], widths=[], rho=[rho0], status="converged",
                    t_final=t, deflated=0)
    if rho0 == 0.0:
        return res
    _check_halving(t, reduce, t_min, list(schedule))
    schedule = set(int(s) for s in schedule)
    rho_prev = rho0
    tol1 = 1.0
    rho_cyc, tol1_cyc = rho0, 1.0  # restart statistic: relative to the cycle's first residual
    k = 1
    level = 0
    t_cur = t
    blocks = []
    colstart = []  # first column of each stored block inside Qbuf
    Qbuf = np.zeros((n, 4 * t), order="F")  # all stored blocks, column-major
    ncols = 0
    Z_prev = None
    pre = precond

    def from_residual(rv, lvl, width):
        if pre is None:
            return split(rv, merged_partition(part, lvl), width)
        return pre.linvT(split(pre.linv(rv), merged_partition(part, lvl), width))

    while rho_prev > tol * rho0 and k < kmax:
        if k == 1:
            cand = from_residual(r, 0, t_cur)
        elif _switch_now(reduce, k, tol1, switch_tol, t_cur, t_min, res.switch_iters, min_gap,
                         schedule):
            level += 1
            t_cur //= 2
            res.switch_iters.append(k)
            cand = from_residual(r, level, t_cur)
            if restart_at_switch:
                res.restart_iters.append(k)
                blocks, colstart, ncols = [], [], 0
                rho_cyc = rho_prev
        elif _restart_now(restart, k, tol1_cyc, restart_every, restart_tol, res.restart_iters, max_restarts):
            res.restart_iters.append(k)
            blocks, colstart, ncols = [], [], 0  # Q is emptied (Section 3)
            rho_cyc = rho_prev
            cand = from_residual(r, level, t_cur)
        elif candidate == "modified-msdo":
            cand = from_residual(r, level, t_cur)
        else:
            cand = Z_prev if pre is None else pre.minv(Z_prev)
        ref2 = np.einsum("ij,ij->j", cand, cand)  # column norms before CGS2 (deflation reference)
        if blocks:
            # Q = all stored blocks, or the last `trunc` of them (Section 3)
            first = 0 if trunc <= 0 else colstart[max(len(blocks) - trunc, 0)]
            cand = a_orthonormalize_against(cand, Qbuf[:, first:ncols], A)
        W = a_orthonormalize_self(cand, A, deflate_tol, ref2=ref2)
        if W is None or W.shape[1] == 0:
            res.status = "breakdown"
            break
        alpha = W.T @ r
        x = x + W @ alpha
        Z = A @ W
        r = r - Z @ alpha
        rho = float(np.linalg.norm(r))
        tol1 = abs(rho - rho_prev) / rho0
        tol1_cyc = abs(rho - rho_prev) / rho_cyc
        rho_prev = rho
        res.rho.append(rho)
        res.widths.append(W.shape[1])
        res.deflated += cand.shape[1] - W.shape[1]
        blocks.append(W)
        colstart.append(ncols)
        if ncols + W.shape[1] > Qbuf.shape[1]:
            grown = np.zeros((n, max(2 * Qbuf.shape[1], ncols + W.shape[1])), order="F")
            grown[:, :ncols] = Qbuf[:, :ncols]
            Qbuf = grown
        Qbuf[:, ncols:ncols + W.shape[1]] = W
        ncols += W.shape[1]
        Z_prev = Z
        if record:
            res.iterates.append(x.copy())
            res.residuals.append(r.copy())
        k += 1
    res.x = x
    res.it = k - 1
    res.t_final = t_cur
    if res.status != "breakdown" and rho_prev > tol * rho0:
        res.status = "not_converged"
    if record:
        res.blocks = blocks
    return res


def cg(A, b, x0=None, tol=1e-8, kmax=100000, record=False):
    """Classical CG (Hestenes-Stiefel), the t = 1 special case (Section 1)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    p = r.copy()
    rr = float(r @ r)
    rho0 = np.sqrt(rr)
    its = []
    k = 0
    while np.sqrt(rr) > tol * rho0 and k < kmax:
        Ap = A @ p
        a = rr / float(p @ Ap)
        x = x + a * p
        r = r - a * Ap
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        k += 1
        if record:
            its.append(x.copy())
    return x, k, its


def true_relres(A, b, x) -> float:
    """||b - A x|| / ||b|| in FP64."""
    return float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))


def memory_formula(t: int, it: int, sit: int) -> int:
    """Stored vectors with one halving at iteration sit+1 (Section 5.2 tables)."""
    return t * sit + (t // 2) * (it - sit)


def flexible_msdo_cg(A, b, part, t, *, x0=None, tol=1e-8, kmax=20000, reduce=REDUCE_NONE, switch_tol=1e-5,
                     t_min=1, min_gap=1, schedule=(), trunc=0, deflate_tol=1e-14,
                     precond: SplitPreconditioner | None = None, record=False, restart=RESTART_NONE,
                     restart_every=0, restart_tol=1e-5, max_restarts=0,
                     restart_at_switch=False) -> EcgResult:
    """Flexibly MSDO-CG (Section 4.4, Algorithm 4; Algorithm 2 without a switch; with a
    split preconditioner, Algorithm 5).

    P_1 = [T^t(r_0)]; at a switch P_k = [T^{t/2}(r_{k-1})]; otherwise
    P_k = [T(r_{k-1})] + P_{k-1} diag(beta_k) with beta_k = -V_{k-1}^T r_{k-1} and
    V_{k-1} = A P_{k-1} (eq. (pk)).  P_k is A-orthonormalised against the stored blocks and
    against itself, then alpha_k = P_k^T r_{k-1}, x_k = x_{k-1} + P_k alpha_k,
    r_k = r_{k-1} - V_k alpha_k.  Preconditioned (Algorithm 5):
    beta_k = -V_{k-1}^T (M^{-1} r_{k-1}) and the split term is L^{-T}[T(L^{-1} r_{k-1})].
    Blocks keep t columns (a deflated column stays a zero column), so column j of P_{k-1}
    always pairs with subdomain j.  Restarts (Section 3) as in ``flexible_sre_cg2``: Q is
    emptied and P_k = [T(r_{k-1})] without the beta term.
    """
    b = np.asarray(b, dtype=np.float64)
    part = np.asarray(part)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    rho0 = float(np.linalg.norm(r))
    res = EcgResult(x=x, it=0, switch_iters=[], widths=[], rho=[rho0], status="converged",
                    t_final=t, deflated=0)
    if rho0 == 0.0:
        return res
    _check_halving(t, reduce, t_min, list(schedule))
    schedule = set(int(s) for s in schedule)
    pre = precond
    rho_prev, tol1, k, level, t_cur = rho0, 1.0, 1, 0, t
    rho_cyc, tol1_cyc = rho0, 1.0
    blocks = []
    P_prev = V_prev = None

    def split_term(rv, lvl, width):
        if pre is None:
            return split(rv, merged_partition(part, lvl), width)
        return pre.linvT(split(pre.linv(rv), merged_partition(part, lvl), width))

    while rho_prev > tol * rho0 and k < kmax:
        if k == 1:
            cand = split_term(r, 0, t_cur)
        elif _switch_now(reduce, k, tol1, switch_tol, t_cur, t_min, res.switch_iters, min_gap, schedule):
            level += 1
            t_cur //= 2
            res.switch_iters.append(k)
            cand = split_term(r, level, t_cur)
            if restart_at_switch:
                res.restart_iters.append(k)
                blocks = []
                rho_cyc = rho_prev
        elif _restart_now(restart, k, tol1_cyc, restart_every, restart_tol, res.restart_iters, max_restarts):
            res.restart_iters.append(k)
            blocks = []
            rho_cyc = rho_prev
            cand = split_term(r, level, t_cur)
        else:
            rr = r if pre is None else pre.minv(r)
            beta = -(V_prev.T @ rr)
            cand = split_term(r, level, t_cur) + P_prev * beta[None, :]
        ref2 = np.einsum("ij,ij->j", cand, cand)  # column norms before CGS2 (deflation reference)
        if record:
            res.candidates.append(cand.copy())
        active = blocks if trunc <= 0 else blocks[-trunc:]
        if active:
            cand = a_orthonormalize_against(cand, np.hstack(active), A)
        P = a_orthonormalize_self(cand, A, deflate_tol, keep_width=True, ref2=ref2)
        live = 0 if P is None else int(np.count_nonzero(np.any(P != 0.0, axis=0)))
        if P is None or live == 0:
            res.status = "breakdown"
            break
        V = A @ P
        alpha = P.T @ r
        x = x + P @ alpha
        r = r - V @ alpha
        rho = float(np.linalg.norm(r))
        tol1 = abs(rho - rho_prev) / rho0
        tol1_cyc = abs(rho - rho_prev) / rho_cyc
        rho_prev = rho
        res.rho.append(rho)
        res.widths.append(live)
        res.deflated += t_cur - live  # every MSDO candidate has t_cur fresh columns
        blocks.append(P)
        P_prev, V_prev = P, V
        if record:
            res.iterates.append(x.copy())
            res.residuals.append(r.copy())
        k += 1
    res.x = x
    res.it = k - 1
    res.t_final = t_cur
    if res.status != "breakdown" and rho_prev > tol * rho0:
        res.status = "not_converged"
    if record:
        res.blocks = blocks
    return res
