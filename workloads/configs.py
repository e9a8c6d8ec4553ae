"""The five synthetic workloads (and scaled-down variants for fast tests).

Each stands in for the paper's FreeFem++ diffusion matrices, which are not
available: a 5-point Poisson problem, 2D and 3D jumping-coefficient finite
volumes, and 3D anisotropic finite differences.  Every array is produced from
numpy's PCG64 generator with a fixed seed.

==========  ================================================================
name        workload
==========  ================================================================
poisson64   5-point Poisson on 64x64, t=8 from 2x4 boxes, no reduction of t
jump2d512   2D two-point FV, 512x512, log10 k ~ U(-3,3) on 32x32-cell blocks,
            t=32 from 4x8 boxes, one halving at switchTol 1e-5
aniso3d128  7-point FD on 128^3 with (x, y, z) coefficients (1, 50, 0.01),
            t in {16, 32, 64} from 2x2x(t/4) boxes
jump3d160   3D two-point FV on 160^3, checkerboard 1/1e6 on 20^3 blocks with
            10% of blocks at 1e-3, t=64 halved repeatedly down to 8
learn2d256  2D two-point FV on 256x256, log10 k ~ U(-3,3) on 16x16 blocks,
            operator seed s, t=16 from 4x4 boxes (learned preconditioner)
==========  ================================================================
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .diffusion import CSR, checker_field_3d, fd_operator, fv_operator, jump_field_2d, rhs_uniform
from .partition import box_partition

CONFIG_NAMES = ("poisson64", "jump2d512", "aniso3d128", "jump3d160", "learn2d256")

# reduction rules (mirrors the C ABI enum values)
REDUCE_NONE = 0
REDUCE_ONCE = 1
REDUCE_REPEAT = 2
REDUCE_SCHEDULE = 3


@dataclass
class Problem:
    name: str
    A: CSR
    b: np.ndarray
    part: np.ndarray
    t: int
    grid: tuple  # cells along (x, y[, z])
    reduce: int = REDUCE_NONE
    switch_tol: float = 1e-5
    t_min: int = 1
    tol: float = 1e-8
    kmax: int = 20000
    # relative tolerance of each inner solve of the FP32 form with FP64 refinement: how far
    # one FP32 solve is driven before the FP64 residual is recomputed
    fp32_inner_tol: float = 1e-4
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.n


def config(name: str, t: int | None = None, seed: int | None = None, scale: int = 1) -> Problem:
    """Build a workload by name.

    t: subdomain count where the workload allows a choice (aniso3d128).
    seed: operator seed for learn2d256.
    scale: divide every grid dimension by this factor (fast tests); the box
      layout and block counts are kept, block sizes shrink with the grid.
    """
    if name == "poisson64":
        nx = ny = 64 // scale
        A = fd_operator((ny, nx), (1.0, 1.0))
        part = box_partition((nx, ny), (2, 4))
        return Problem(name, A, rhs_uniform(A.n, 0), part, 8, (nx, ny))
    if name == "jump2d512":
        nx = ny = 512 // scale
        k = jump_field_2d(nx, ny, 32 // scale, seed=1)
        A = fv_operator(k)
        part = box_partition((nx, ny), (4, 8))
        return Problem(name, A, rhs_uniform(A.n, 2), part, 32, (nx, ny), reduce=REDUCE_ONCE,
                       switch_tol=1e-5, t_min=16)
    if name == "aniso3d128":
        t = 32 if t is None else int(t)
        if t not in (16, 32, 64):
            raise ValueError("aniso3d128 takes t in {16, 32, 64}")
        m = 128 // scale
        A = fd_operator((m, m, m), (0.01, 50.0, 1.0))  # (z, y, x) coefficients
        part = box_partition((m, m, m), (2, 2, t // 4))
        return Problem(name, A, rhs_uniform(A.n, 3), part, t, (m, m, m), reduce=REDUCE_ONCE,
                       switch_tol=1e-5, t_min=t // 2)
    if name == "jump3d160":
        m = 160 // scale
        k = checker_field_3d(m, 20 // scale, seed=4)
        A = fv_operator(k)
        part = box_partition((m, m, m), (4, 4, 4))
        return Problem(name, A, rhs_uniform(A.n, 5), part, 64, (m, m, m), reduce=REDUCE_REPEAT,
                       switch_tol=1e-5, t_min=8, fp32_inner_tol=1e-5)
    if name == "learn2d256":
        s = 0 if seed is None else int(seed)
        nx = ny = 256 // scale
        k = jump_field_2d(nx, ny, max(16 // scale, 1), seed=s)
        A = fv_operator(k)
        part = box_partition((nx, ny), (4, 4))
        return Problem(name, A, rhs_uniform(A.n, 10 ** 6 + s), part, 16, (nx, ny),
                       extra={"k": k, "seed": s})
    raise KeyError(name)
