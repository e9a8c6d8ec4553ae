"""Preconditioners for the oracle (TEST INFRASTRUCTURE ONLY).

* Block-Jacobi incomplete Cholesky with zero fill (Section 5.3): A restricted to
  each subdomain, couplings between subdomains dropped; each diagonal block is
  factored L_i L_i^T keeping exactly the sparsity of its lower triangle.  The
  textbook IC(0) recurrence, row by row in the matrix ordering:
      L_ij = (a_ij - sum_{k<j} L_ik L_jk) / L_jj   for (i, j) in the pattern, j < i
      L_ii = sqrt(a_ii - sum_{k<i} L_ik^2)
  with the sums running over the common pattern only.
* Block-Jacobi Cholesky (Section 5.3, eq. (cholprec)): the same diagonal blocks factored
  exactly, A_i = L_i L_i^T (LAPACK Cholesky of each dense block), so M is the block
  diagonal of A itself.  The blocks are independent of t (the paper uses 64 or 128 of
  them for every t; the t subdomains are unions of consecutive blocks).
* A factorised approximate inverse M^{-1} = G G^T, for which L^{-1} = G^T and
  L^{-T} = G in the split-preconditioned recurrences (Section 4.5, eq. (zsre2)).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from .ecg import SplitPreconditioner


def block_diagonal_part(A: sp.csr_matrix, part: np.ndarray) -> sp.csr_matrix:
    """A with every entry a_ij, part[i] != part[j], removed."""
    A = sp.csr_matrix(A)
    coo = A.tocoo()
    keep = part[coo.row] == part[coo.col]
    return sp.csr_matrix((coo.data[keep], (coo.row[keep], coo.col[keep])), shape=A.shape)


def ic0(A: sp.csr_matrix) -> sp.csr_matrix:
    """IC(0) factor L (lower triangular CSR, same pattern as tril(A)).

    Raises ValueError on a non-positive pivot.
    """
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    low = sp.tril(A, format="csr")
    low.sort_indices()
    rows = []  # per row: dict col -> L value
    for i in range(n):
        cols = low.indices[low.indptr[i]:low.indptr[i + 1]]
        vals = low.data[low.indptr[i]:low.indptr[i + 1]]
        Li = {}
        for c, a in zip(cols, vals):
            if c == i:
                continue
            s = a
            Lc = rows[c]
            for k, lik in Li.items():
                if k < c and k in Lc:
                    s -= lik * Lc[k]
            Li[c] = s / Lc[c]
        d = vals[cols == i]
        if d.size != 1:
            raise ValueError("missing diagonal")
        piv = d[0] - sum(v * v for k, v in Li.items())
        if not piv > 0:
            raise ValueError(f"IC(0) pivot not positive at row {i}")
        Li[i] = np.sqrt(piv)
        rows.append(Li)
    indptr = np.zeros(n + 1, dtype=np.int64)
    ind = []
    dat = []
    for i, Li in enumerate(rows):
        ks = sorted(Li)
        ind.extend(ks)
        dat.extend(Li[k] for k in ks)
        indptr[i + 1] = len(ind)
    return sp.csr_matrix((np.array(dat), np.array(ind, dtype=np.int64), indptr), shape=(n, n))


def _tri_solve(T, X, lower):
    X = np.asarray(X, dtype=np.float64)
    return spl.spsolve_triangular(sp.csr_matrix(T), X, lower=lower)


def bj_ic0_preconditioner(A, part) -> tuple[SplitPreconditioner, sp.csr_matrix]:
    """Block-Jacobi IC(0) on the subdomains of ``part``: (preconditioner, L)."""
    L = ic0(block_diagonal_part(A, np.asarray(part)))
    LT = sp.csr_matrix(L.T)
    pre = SplitPreconditioner(lambda X: _tri_solve(L, X, True), lambda X: _tri_solve(LT, X, False))
    return pre, L


def block_cholesky(A, blocks) -> sp.csr_matrix:
    """Exact Cholesky factor of every diagonal block of A (blocks[i] = block of row i):
    the lower-triangular L with L L^T = blockdiag(A), rows in the matrix ordering."""
    A = sp.csr_matrix(A)
    blocks = np.asarray(blocks)
    n = A.shape[0]
    rows, cols, vals = [], [], []
    for g in np.unique(blocks):
        idx = np.flatnonzero(blocks == g)
        Ag = A[idx][:, idx].toarray()
        Lg = np.linalg.cholesky(Ag)  # raises LinAlgError unless the block is SPD
        r, c = np.nonzero(np.tril(Lg))
        rows.append(idx[r])
        cols.append(idx[c])
        vals.append(Lg[r, c])
    L = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    L.sort_indices()
    return L


def bj_chol_preconditioner(A, blocks) -> tuple[SplitPreconditioner, sp.csr_matrix]:
    """Block-Jacobi exact Cholesky on the blocks of ``blocks``: (preconditioner, L)."""
    L = block_cholesky(A, blocks)
    LT = sp.csr_matrix(L.T)
    pre = SplitPreconditioner(lambda X: _tri_solve(L, X, True), lambda X: _tri_solve(LT, X, False))
    return pre, L


def factor_preconditioner(G) -> SplitPreconditioner:
    """M^{-1} = G G^T: L^{-1} X = G^T X and L^{-T} X = G X."""
    G = sp.csr_matrix(G)
    GT = sp.csr_matrix(G.T)
    return SplitPreconditioner(lambda X: GT @ X, lambda X: G @ X)
