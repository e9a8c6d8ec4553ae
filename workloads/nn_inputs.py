"""Inputs of the learned preconditioner: stencil layout and initial network parameters.

Both are inputs (a data layout and seeded random numbers), not part of the method.
"""

from __future__ import annotations

import numpy as np

NF, NH, NO = 7, 32, 3
NPARAM = NH * NF + NH + NH * NH + NH + NO * NH + NO  # 1411


def stencil5(csr, nx: int) -> np.ndarray:
    """(5, n) array of a 5-point operator in natural order: diagonal, west, east, south,
    north coefficient of every row (0 where the neighbour is outside the grid)."""
    n = csr.n
    rows = np.repeat(np.arange(n), np.diff(csr.rowptr))
    off = csr.colind.astype(np.int64) - rows
    out = np.zeros((5, n))
    for k, d in enumerate((0, -1, 1, -nx, nx)):
        m = off == d
        out[k, rows[m]] = csr.vals[m]
    return out


def init_params(seed: int) -> np.ndarray:
    """Flat parameters W1 (32x7), b1, W2 (32x32), b2, W3 (3x32), b3: the hidden weights are
    N(0, 1/fan_in) from numpy's PCG64(seed); biases and the last layer are zero, so the
    untrained network outputs 0 (the Jacobi factor)."""
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal((NH, NF)) / np.sqrt(NF)
    w2 = rng.standard_normal((NH, NH)) / np.sqrt(NH)
    return np.concatenate([w1.ravel(), np.zeros(NH), w2.ravel(), np.zeros(NH), np.zeros(NO * NH), np.zeros(NO)])
