"""Coplanar interpolation I^H from coarse nodes to a fine skeleton node
(paper sec. 3.1 eq. mlcdiscr and sec. 4.1 eq. mlcfulldiscr).

The paper fixes only that the interpolation points are coplanar with the
target, that the stencil radius is b and that the order is q_I (b = 2 -> 6,
b = 3 -> 8, sec. 7.1); the operator itself is deferred to an earlier paper.
Reading used: tensor-product 1-D Lagrange interpolation in the plane of the
patch face through the target node, on the 2b+2 coarse nodes U0-b .. U0+b+1
per in-plane axis, with U0 = floor(g_a / Nref); degree 2b+1, order 2b+2 =
q_I.  A node that falls on a coarse node (theta = 0) takes that node's
value.  Parity unpinned against the paper's own operator (only its order is
pinned by tests).
"""
import numpy as np

from .geometry import NREF


def lagrange_weights(b, theta):
    """w_k(theta), k = -b..b+1: Lagrange basis on the integer nodes
    -b..b+1 evaluated at theta.  Returns shape (2b+2,)."""
    nodes = np.arange(-b, b + 2, dtype=np.float64)
    w = np.ones(len(nodes))
    for k, xk in enumerate(nodes):
        for m, xm in enumerate(nodes):
            if m != k:
                w[k] *= (theta - xm) / (xk - xm)
    return w


def normal_axis(g, n):
    """The axis of the face plane used for a skeleton node g: the lowest
    axis d with g_d divisible by n (any choice gives the same value)."""
    for d in range(3):
        if g[d] % n == 0:
            return d
    raise ValueError("not a skeleton node")


def stencil(g, n, b, d=None):
    """Coarse interpolation stencil of the skeleton node g in the plane of
    normal axis d (default: normal_axis).  Returns (coarse_pts, weights):
    coarse_pts has shape (2b+2, 2b+2, 3) (coarse node indices), weights
    (2b+2, 2b+2).  Coarse node c corresponds to the fine node Nref c."""
    if d is None:
        d = normal_axis(g, n)
    a0, a1 = [a for a in range(3) if a != d]
    U0 = [g[a0] // NREF, g[a1] // NREF]
    th = [(g[a0] - NREF * U0[0]) / NREF, (g[a1] - NREF * U0[1]) / NREF]
    w0 = lagrange_weights(b, th[0])
    w1 = lagrange_weights(b, th[1])
    ks = np.arange(-b, b + 2)
    pts = np.zeros((len(ks), len(ks), 3), dtype=np.int64)
    pts[:, :, d] = g[d] // NREF
    pts[:, :, a0] = (U0[0] + ks)[:, None]
    pts[:, :, a1] = (U0[1] + ks)[None, :]
    return pts, w0[:, None] * w1[None, :]
