"""Mehrstellen discretisations of the 3-D Laplacian (paper sec. 2, eq. for
the discrete Laplacian; appendix A.1 gives the coefficients).

The stencil acts on the 3x3x3 neighbourhood of a node; the weight of the
offset s is b[k]/h^2 where k is the number of non-zero components of s.
L19 (q = 4) and L27 (q = 6) share the correction constant C2 = 1/12 (sec. 2).
"""
import numpy as np

# appendix A.1: b_0..b_3 for the 19-point and the 27-point operator
_B = {
    4: (-4.0, 1.0 / 3.0, 1.0 / 6.0, 0.0),
    6: (-64.0 / 15.0, 7.0 / 15.0, 1.0 / 10.0, 1.0 / 30.0),
}
# a plain 7-point Laplacian; used only to pin the DGF solver against
# Watson's lattice Green's function value (not part of the method)
_B7 = (-6.0, 1.0, 0.0, 0.0)

C2 = 1.0 / 12.0


def stencil_b(Q):
    """b_0..b_3 of the order-Q Mehrstellen operator (Q=4: L19, Q=6: L27).
    Q=2 selects the 7-point operator (test use only)."""
    if Q == 2:
        return _B7
    return _B[Q]


def stencil_weights(Q):
    """3x3x3 array a[s+1] = b_{|s|} (h = 1)."""
    b = stencil_b(Q)
    a = np.empty((3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                nz = (i != 1) + (j != 1) + (k != 1)
                a[i, j, k] = b[nz]
    return a


def apply_laplacian(u, Q, h=1.0):
    """Delta^h u on the nodes of u that have a full 3x3x3 neighbourhood.

    Returns an array two nodes shorter along every axis.  Definition:
    (Delta^h u)[g] = sum_{s in [-1,1]^3} a_s u[g+s] / h^2.
    """
    a = stencil_weights(Q)
    n0, n1, n2 = u.shape
    out = np.zeros((n0 - 2, n1 - 2, n2 - 2))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                if a[i, j, k] != 0.0:
                    out += a[i, j, k] * u[i:i + n0 - 2, j:j + n1 - 2, k:k + n2 - 2]
    return out / (h * h)


def symbol(Q, c0, c1, c2):
    """Eigenvalue of the h=1 stencil on the separable cosine / sine mode with
    per-axis cosines c0, c1, c2:
        b0 + 2 b1 (c0+c1+c2) + 4 b2 (c0c1+c0c2+c1c2) + 8 b3 c0c1c2.
    (Each axis factor sin(theta(m+s)) + sin(theta(m-s)) = 2 sin(theta m) cos(theta s).)
    """
    b = stencil_b(Q)
    return (b[0] + 2.0 * b[1] * (c0 + c1 + c2)
            + 4.0 * b[2] * (c0 * c1 + c0 * c2 + c1 * c2)
            + 8.0 * b[3] * c0 * c1 * c2)


def _shift(u, d, k):
    """u[g + k e_d] with zeros beyond the array (f extended by zero)."""
    out = np.zeros_like(u)
    n = u.shape[d]
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    if k >= 0:
        src[d] = slice(k, n)
        dst[d] = slice(0, n - k)
    else:
        src[d] = slice(0, n + k)
        dst[d] = slice(-k, n)
    out[tuple(dst)] = u[tuple(src)]
    return out


def sixth_order_rhs(f):
    """The modified right-hand side of sec. 2 eq. msCorr for the 27-point
    operator (q = 6), with the h^4 operator read off its truncation error in
    appendix A.1:
        f~ = f + C2 h^2 (Delta f)_4 + (h^4 / 360) (Delta^2 + 2 (d_xxyy + d_yyzz + d_zzxx)) f,
    (Delta f)_4 the fourth-order central differences along each axis, the h^4
    term second-order differences (d_dd d_ee f as products of second
    differences).  Then Delta^h phi = f~ + O(h^6), so G^h * f~ is sixth-order
    accurate with no final correction.  Every difference is in units of h (the
    result does not depend on h).  f is extended by zero past the array; it
    must vanish within two nodes of the array's faces so that f~ vanishes on
    them."""
    f = np.asarray(f, dtype=np.float64)
    for d in range(3):
        for k in (0, 1, 2, -1, -2, -3):
            if np.any(np.take(f, k, axis=d) != 0.0):
                raise ValueError("f must vanish within two nodes of the faces")
    return sixth_order_rhs_stencil(f)


def sixth_order_rhs_stencil(f):
    """The differences of sixth_order_rhs on every node, f extended by zero
    (exact at the nodes two or more from the array's faces for any f)."""
    d2 = [_shift(f, d, 1) - 2.0 * f + _shift(f, d, -1) for d in range(3)]
    lap4 = sum((-_shift(f, d, 2) + 16.0 * _shift(f, d, 1) - 30.0 * f + 16.0 * _shift(f, d, -1) - _shift(f, d, -2))
               / 12.0 for d in range(3))
    quart = sum(_shift(d2[d], d, 1) - 2.0 * d2[d] + _shift(d2[d], d, -1) for d in range(3))
    mixed = sum(_shift(d2[d], e, 1) - 2.0 * d2[d] + _shift(d2[d], e, -1) for d in range(3) for e in range(d + 1, 3))
    return f + C2 * lap4 + (quart + 4.0 * mixed) / 360.0
