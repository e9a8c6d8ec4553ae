"""Structured-grid diffusion operators (symmetric positive definite, CSR).

Ordering is natural lexicographic with x fastest: cell (x, y[, z]) has index
x + nx*y (+ nx*ny*z).  Grid spacing factors are dropped (they only scale A).
Dirichlet boundaries are eliminated, so every operator is SPD.

Two discretisations are provided:

* ``fd_operator``: constant-coefficient finite differences, diagonal
  2*sum(c_axis), off-diagonal -c_axis for every neighbour inside the grid
  (the 5-point Poisson matrix is ``fd_operator((ny, nx), (1, 1))``).
* ``fv_operator``: cell-centred two-point finite volumes with a per-cell
  coefficient k.  The transmissibility of an interior face is the harmonic
  mean 2 k_a k_b / (k_a + k_b); a boundary face (Dirichlet at distance h/2)
  contributes 2 k_a to the diagonal.

Columns inside each CSR row are sorted ascending.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    """Sparse matrix in compressed-sparse-row form.

    rowptr: int64[n+1]; colind: int32[nnz]; vals: float64[nnz].
    """

    n: int
    rowptr: np.ndarray
    colind: np.ndarray
    vals: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.vals, self.colind, self.rowptr), shape=(self.n, self.n))

    def diagonal(self) -> np.ndarray:
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        d = np.zeros(self.n)
        m = rows == self.colind
        d[rows[m]] = self.vals[m]
        return d


def _strides(shape):
    """Strides (in cells) of each axis for a C-ordered shape (slowest first)."""
    st = []
    acc = 1
    for s in reversed(shape):
        st.append(acc)
        acc *= s
    return list(reversed(st))


def _assemble(shape, diag, offdiag):
    """Build CSR from per-axis neighbour couplings.

    shape: grid shape, slowest axis first (e.g. (nz, ny, nx)).
    diag: float64 array of the grid shape.
    offdiag: list over axes (same order as shape) of arrays of shape with that
      axis shortened by one: coupling between cell c and c + e_axis (the value
      stored is the matrix entry, i.e. already negative).
    """
    d = len(shape)
    n = int(np.prod(shape))
    strides = _strides(shape)
    # Candidate columns in ascending order: -axis0 ... -axis(d-1), 0, +axis(d-1) ... +axis0
    offs = [-strides[a] for a in range(d)] + [0] + [strides[a] for a in reversed(range(d))]
    ncand = len(offs)
    vals = np.zeros((n, ncand))
    mask = np.zeros((n, ncand), dtype=bool)
    vals[:, d] = diag.reshape(-1)
    mask[:, d] = True
    for a in range(d):
        od = offdiag[a]
        # coupling with +axis neighbour: cells with coordinate < shape[a]-1
        plus = np.zeros(shape)
        sl_lo = [slice(None)] * d
        sl_lo[a] = slice(0, shape[a] - 1)
        plus[tuple(sl_lo)] = od
        pmask = np.zeros(shape, dtype=bool)
        pmask[tuple(sl_lo)] = True
        # coupling with -axis neighbour: cells with coordinate > 0
        minus = np.zeros(shape)
        sl_hi = [slice(None)] * d
        sl_hi[a] = slice(1, shape[a])
        minus[tuple(sl_hi)] = od
        mmask = np.zeros(shape, dtype=bool)
        mmask[tuple(sl_hi)] = True
        jm = a  # position of -axis a
        jp = ncand - 1 - a  # position of +axis a
        vals[:, jm] = minus.reshape(-1)
        mask[:, jm] = mmask.reshape(-1)
        vals[:, jp] = plus.reshape(-1)
        mask[:, jp] = pmask.reshape(-1)
    idx = np.arange(n, dtype=np.int64)[:, None] + np.asarray(offs, dtype=np.int64)[None, :]
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colind = idx[mask].astype(np.int32)
    v = vals[mask].astype(np.float64)
    return CSR(n, rowptr, colind, v)


def fd_operator(shape, coeffs) -> CSR:
    """Constant-coefficient 2d+1-point finite-difference operator.

    shape: grid shape slowest axis first, e.g. (ny, nx) or (nz, ny, nx).
    coeffs: per-axis coefficient in the same order as ``shape``.
    """
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    diag = np.full(shape, 2.0 * float(sum(coeffs)))
    off = []
    for a in range(d):
        s = list(shape)
        s[a] -= 1
        off.append(np.full(s, -float(coeffs[a])))
    return _assemble(shape, diag, off)


def fv_operator(k: np.ndarray) -> CSR:
    """Two-point flux finite volumes for -div(k grad u) with Dirichlet walls.

    k: positive per-cell coefficient, shape = grid shape slowest axis first.
    """
    k = np.asarray(k, dtype=np.float64)
    shape = k.shape
    d = k.ndim
    diag = np.zeros(shape)
    off = []
    for a in range(d):
        lo = [slice(None)] * d
        hi = [slice(None)] * d
        lo[a] = slice(0, shape[a] - 1)
        hi[a] = slice(1, shape[a])
        ka = k[tuple(lo)]
        kb = k[tuple(hi)]
        tr = 2.0 * ka * kb / (ka + kb)
        diag[tuple(lo)] += tr
        diag[tuple(hi)] += tr
        off.append(-tr)
        # boundary faces on both walls of this axis
        first = [slice(None)] * d
        last = [slice(None)] * d
        first[a] = 0
        last[a] = shape[a] - 1
        diag[tuple(first)] += 2.0 * k[tuple(first)]
        diag[tuple(last)] += 2.0 * k[tuple(last)]
    return _assemble(shape, diag, off)


def jump_field_2d(nx: int, ny: int, block: int, seed: int, lo: float = -3.0, hi: float = 3.0) -> np.ndarray:
    """Piecewise-constant coefficient on block x block cells, log10 k ~ U(lo, hi).

    Returns k with shape (ny, nx).  The block values are drawn in row-major
    block order (block-row y slowest) from numpy's PCG64 with ``seed``.
    """
    nbx, nby = nx // block, ny // block
    rng = np.random.default_rng(seed)
    logk = rng.uniform(lo, hi, size=(nby, nbx))
    kb = 10.0 ** logk
    return np.repeat(np.repeat(kb, block, axis=0), block, axis=1)


def checker_field_3d(n: int, block: int, seed: int, high: float = 1e6, low: float = 1e-3,
                     frac_low: float = 0.1) -> np.ndarray:
    """3D checkerboard of 1 / ``high`` on block^3 cells; a random ~10% of the
    blocks (chosen without replacement) are set to ``low``.  Shape (n, n, n)."""
    nb = n // block
    bz, by, bx = np.meshgrid(np.arange(nb), np.arange(nb), np.arange(nb), indexing="ij")
    kb = np.where((bx + by + bz) % 2 == 0, 1.0, high)
    rng = np.random.default_rng(seed)
    nlow = int(round(frac_low * nb ** 3))
    pick = rng.choice(nb ** 3, size=nlow, replace=False)
    kb.reshape(-1)[pick] = low
    return np.repeat(np.repeat(np.repeat(kb, block, axis=0), block, axis=1), block, axis=2)


def rhs_uniform(n: int, seed: int) -> np.ndarray:
    """Right-hand side b ~ U(-1, 1)^n from numpy's PCG64 with ``seed``."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)
