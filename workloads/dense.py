"""Tiny dense SPD test matrices (for exhaustive checks of the oracle)."""

from __future__ import annotations

import numpy as np

from .diffusion import CSR


def random_spd(n: int, kappa: float, seed: int) -> np.ndarray:
    """Dense SPD matrix with eigenvalues log-spaced in [1, kappa].

    A = V diag(lambda) V^T with V a Haar-random orthogonal matrix drawn from
    numpy's PCG64 with ``seed``; the result is symmetrised exactly.
    """
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n))
    v, r = np.linalg.qr(g)
    v = v * np.sign(np.diag(r))[None, :]
    lam = np.logspace(0.0, np.log10(kappa), n)
    a = (v * lam[None, :]) @ v.T
    return 0.5 * (a + a.T)


def dense_to_csr(a: np.ndarray, drop_zeros: bool = False) -> CSR:
    """Store a dense matrix as CSR (all entries kept unless ``drop_zeros``)."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    if drop_zeros:
        mask = a != 0.0
    else:
        mask = np.ones_like(a, dtype=bool)
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    cols = np.nonzero(mask)[1].astype(np.int32)
    return CSR(n, rowptr, cols, a[mask].copy())
