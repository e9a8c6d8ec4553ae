"""High-precision, basis-free definitions of the ECG iterates (TEST INFRASTRUCTURE ONLY).

Used on tiny inputs (n <= ~48) to pin ``oracle.ecg`` with no code in common:
everything here is mpmath at 50 significant digits, with the subspaces
defined directly rather than through the solver's block recurrences.

* ``krylov_projection``: the Petrov-Galerkin iterate of Section 2,
  x_k = x_0 + V (V^T A V)^{-1} V^T r_0, where the columns of V are the
  monomial block basis T^t(r_0), A T^t(r_0), ..., A^{k-1} T^t(r_0) of the
  enlarged Krylov subspace K_{k,t}(A, r_0) (Section 1).
* ``recursion_projection``: the same Galerkin iterate on the subspaces that
  Algorithm 3 builds when it switches: S_1 = span T^t(r_0); a regular step
  adds A times the A-orthogonal complement of S_{k-1} in S_k; a switch step
  adds span T^{t/2}(r_k), with r_k the Galerkin residual on S_k.
* ``msdo_projection``: the Galerkin iterates of MSDO-CG / modified MSDO-CG, on the
  modified subspace span{T(r_0), ..., T(r_{k-1})} of Section 2.2 (r_j the Galerkin
  residual on the previous subspace; after a switch the split uses t/2 merged subdomains).
* ``cg_iterates``: classical CG in 50 digits (the t = 1 case).
"""

from __future__ import annotations

import mpmath as mp
import numpy as np

DPS = 50


def _mat(a):
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    return mp.matrix([[mp.mpf(float(v)) for v in row] for row in a])


def _to_np(m):
    return np.array([[float(m[i, j]) for j in range(m.cols)] for i in range(m.rows)])


def _hcat(blocks):
    rows = blocks[0].rows
    cols = sum(b.cols for b in blocks)
    out = mp.matrix(rows, cols)
    c = 0
    for b in blocks:
        for j in range(b.cols):
            for i in range(rows):
                out[i, c] = b[i, j]
            c += 1
    return out


def _split(v, part, t):
    n = v.rows
    out = mp.matrix(n, t)
    for i in range(n):
        out[i, int(part[i])] = v[i, 0]
    return out


def _galerkin(A, V, r0):
    """V (V^T A V)^{-1} V^T r0 in high precision (V with independent columns)."""
    G = V.T * A * V
    rhs = V.T * r0
    return V * mp.lu_solve(G, rhs)


def _a_orth_basis(A, V, prev=None, drop=mp.mpf("1e-30")):
    """A-orthonormal basis of span(V) minus span(prev) by MGS (prev is A-orthonormal)."""
    cols = []
    for j in range(V.cols):
        v = V[:, j]
        for q in ([prev[:, i] for i in range(prev.cols)] if prev is not None else []) + cols:
            v = v - q * (q.T * A * v)[0, 0]
        for q in ([prev[:, i] for i in range(prev.cols)] if prev is not None else []) + cols:
            v = v - q * (q.T * A * v)[0, 0]
        nv = mp.sqrt((v.T * A * v)[0, 0])
        scale = mp.sqrt((V[:, j].T * A * V[:, j])[0, 0])
        if nv > drop * scale:
            cols.append(v / nv)
    if not cols:
        return mp.matrix(V.rows, 0) if False else None
    return _hcat(cols)


def krylov_projection(A, b, part, t, k, x0=None):
    """Galerkin iterate on x0 + K_{k,t}(A, r0) (float64 result)."""
    with mp.workdps(DPS):
        Am = _mat(A)
        x0m = _mat(np.zeros(len(b)) if x0 is None else x0)
        r0 = _mat(b) - Am * x0m
        blk = _split(r0, part, t)
        blocks = [blk]
        for _ in range(1, k):
            blocks.append(Am * blocks[-1])
        V = _hcat(blocks)
        x = x0m + _galerkin(Am, V, r0)
        return _to_np(x)[:, 0]


def recursion_projection(A, b, part, t, k_total, switch_iters=(), x0=None):
    """Galerkin iterates x_1..x_k_total on the subspaces Algorithm 3 builds.

    switch_iters: iterations k at which the added block is T^{t_cur/2}(r_{k-1})
    on the merged partition (part >> number of switches so far).
    Returns a list of float64 iterates.
    """
    switch_iters = set(int(s) for s in switch_iters)
    with mp.workdps(DPS):
        Am = _mat(A)
        x0m = _mat(np.zeros(len(b)) if x0 is None else x0)
        r0 = _mat(b) - Am * x0m
        basis = None  # A-orthonormal basis of S_k
        newest = None  # A-orthonormal basis of S_k (-) S_{k-1}
        t_cur, level = t, 0
        r = r0
        out = []
        for k in range(1, k_total + 1):
            if k == 1:
                cand = _split(r0, part, t_cur)
            elif k in switch_iters:
                level += 1
                t_cur //= 2
                cand = _split(r, np.asarray(part) >> level, t_cur)
            else:
                cand = Am * newest
            newest = _a_orth_basis(Am, cand, basis)
            basis = newest if basis is None else _hcat([basis, newest])
            x = x0m + basis * (basis.T * r0)
            r = _mat(b) - Am * x
            out.append(_to_np(x)[:, 0])
        return out


def msdo_projection(A, b, part, t, k_total, switch_iters=(), x0=None):
    """Galerkin iterates x_1..x_k_total on S_k = span{T(r_0), ..., T(r_{k-1})}."""
    switch_iters = set(int(s) for s in switch_iters)
    with mp.workdps(DPS):
        Am = _mat(A)
        x0m = _mat(np.zeros(len(b)) if x0 is None else x0)
        r0 = _mat(b) - Am * x0m
        basis = None
        t_cur, level = t, 0
        r = r0
        out = []
        for k in range(1, k_total + 1):
            if k in switch_iters:
                level += 1
                t_cur //= 2
            cand = _split(r, np.asarray(part) >> level, t_cur)
            newest = _a_orth_basis(Am, cand, basis)
            basis = newest if basis is None else _hcat([basis, newest])
            x = x0m + basis * (basis.T * r0)
            r = _mat(b) - Am * x
            out.append(_to_np(x)[:, 0])
        return out


def cg_iterates(A, b, k_total, x0=None):
    """Classical CG iterates x_1..x_k_total in 50 digits."""
    with mp.workdps(DPS):
        Am = _mat(A)
        x = _mat(np.zeros(len(b)) if x0 is None else x0)
        r = _mat(b) - Am * x
        p = r.copy()
        rr = (r.T * r)[0, 0]
        out = []
        for _ in range(k_total):
            Ap = Am * p
            a = rr / (p.T * Ap)[0, 0]
            x = x + p * a
            r = r - Ap * a
            rr2 = (r.T * r)[0, 0]
            p = r + p * (rr2 / rr)
            rr = rr2
            out.append(_to_np(x)[:, 0])
        return out


def a_norm_error(A, xstar, x) -> float:
    e = np.asarray(xstar) - np.asarray(x)
    return float(np.sqrt(max(e @ (np.asarray(A) @ e), 0.0)))
