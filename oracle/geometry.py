"""Index boxes and the patch geometry of the fully discrete MLC
(paper sec. 2 notation; sec. 4 first paragraph).

A box is a pair (lo, hi) of integer 3-vectors; it denotes the closed set of
nodes lo <= g <= hi.  Axis order is the array-axis order (0, 1, 2).
"""
import math
from fractions import Fraction

import numpy as np

NREF = 4  # refinement ratio between the fine and the coarse grid (sec. 2)


def box(lo, hi):
    return (np.asarray(lo, dtype=np.int64), np.asarray(hi, dtype=np.int64))


def grow(b, r):
    """G(D, r) = [l - r, u + r] (sec. 2)."""
    return (b[0] - r, b[1] + r)


def coarsen(b):
    """C(D) = [floor(l / Nref), ceil(u / Nref)] (sec. 2)."""
    return (np.floor_divide(b[0], NREF), -np.floor_divide(-b[1], NREF))


def contains(b, g):
    """Membership of node(s) g (shape (..., 3)) in the closed box b."""
    g = np.asarray(g)
    return np.all((g >= b[0]) & (g <= b[1]), axis=-1)


def margin(radius, n):
    """Half-margin ceil((radius - 1) n / 2) of the localisation region
    Omega_{R,i,radius} = G(Omega_{R,i}, margin) (sec. 4)."""
    r = Fraction(radius).limit_denominator(10_000)
    return int(math.ceil((r - 1) * n / 2))


def patch_box(i, n):
    """Omega_{R,i}^h = n i + [0, n]^3 (sec. 4)."""
    i = np.asarray(i, dtype=np.int64)
    return (n * i, n * i + n)


def patch_indices(N, n):
    """All patch indices i covering [0, N]^3, as an (npatch, 3) array in
    C order (axis 2 fastest)."""
    m = N // n
    ii = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1)
    return ii.reshape(-1, 3)
