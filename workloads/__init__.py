"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only *generates* inputs (sparse SPD diffusion operators in CSR
form, right-hand sides and subdomain partitions).  It contains none of the
solver's arithmetic, so both the CPU oracle and the GPU path may import it
without sharing any part of the method.
"""

from .diffusion import (  # noqa: F401
    CSR,
    fd_operator,
    fv_operator,
    jump_field_2d,
    checker_field_3d,
    rhs_uniform,
)
from .partition import box_partition, morton_box_ids, random_partition  # noqa: F401
from .dense import random_spd, dense_to_csr  # noqa: F401
from .configs import Problem, config, CONFIG_NAMES  # noqa: F401
from .nn_inputs import stencil5, init_params, NPARAM  # noqa: F401
