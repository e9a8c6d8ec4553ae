"""Subdomain partitions for the enlarged Krylov subspace.

A partition is an int32 map ``part[i] in [0, t)`` giving the subdomain of
unknown i (the paper's disjoint index sets delta_1..delta_t, Section 2).

When t is halved, subdomains 2i and 2i+1 (0-based) merge into subdomain i
(Section 4, definition of T^{t/2}), i.e. the merged map is ``part >> 1``.
For box partitions of a grid the box ids are therefore numbered so that the
lowest id bit separates two boxes that are neighbours along one axis: the id
is built from its least significant bit upward, each bit taken from the axis
that still has the most unused bits of its box coordinate (ties go to x, then
y, then z).  Shifting the id right by one then merges pairs of boxes along the
axis that was split last, so repeated halving keeps subdomains compact boxes.
"""

from __future__ import annotations

import numpy as np


def _log2(v: int) -> int:
    b = int(v).bit_length() - 1
    if (1 << b) != v:
        raise ValueError(f"box count {v} is not a power of two")
    return b


def morton_box_ids(boxes_xyz) -> np.ndarray:
    """Box id for every box coordinate.

    boxes_xyz: number of boxes along (x, y[, z]).
    Returns an int array with shape (Bz, By, Bx) (or (By, Bx)) of ids.
    """
    boxes_xyz = [int(b) for b in boxes_xyz]
    d = len(boxes_xyz)
    bits = [_log2(b) for b in boxes_xyz]
    coords = np.meshgrid(*[np.arange(b) for b in reversed(boxes_xyz)], indexing="ij")
    coords = list(reversed(coords))  # coords[a] is the axis-a coordinate (x first)
    ids = np.zeros(coords[0].shape, dtype=np.int64)
    remaining = list(bits)
    taken = [0] * d
    pos = 0
    while any(r > 0 for r in remaining):
        a = max(range(d), key=lambda ax: (remaining[ax], -ax))
        ids |= ((coords[a] >> taken[a]) & 1) << pos
        taken[a] += 1
        remaining[a] -= 1
        pos += 1
    return ids


def box_partition(grid_xyz, boxes_xyz) -> np.ndarray:
    """Partition a grid into equal boxes numbered by ``morton_box_ids``.

    grid_xyz: cells along (x, y[, z]); boxes_xyz: boxes along the same axes.
    Returns int32 part[n] in the grid's lexicographic order (x fastest).
    """
    grid_xyz = [int(g) for g in grid_xyz]
    boxes_xyz = [int(b) for b in boxes_xyz]
    for g, b in zip(grid_xyz, boxes_xyz):
        if g % b:
            raise ValueError("grid size must be a multiple of the box count")
    ids = morton_box_ids(boxes_xyz)
    # per-cell box coordinate along each axis
    axes = [np.arange(g) // (g // b) for g, b in zip(grid_xyz, boxes_xyz)]
    mesh = np.meshgrid(*reversed(axes), indexing="ij")  # slowest axis first
    part = ids[tuple(mesh)]
    return part.reshape(-1).astype(np.int32)


def random_partition(n: int, t: int, seed: int) -> np.ndarray:
    """Random partition of n unknowns into t non-empty subdomains."""
    if t > n:
        raise ValueError("t must not exceed n")
    rng = np.random.default_rng(seed)
    part = np.concatenate([np.arange(t), rng.integers(0, t, size=n - t)])
    rng.shuffle(part)
    return part.astype(np.int32)
