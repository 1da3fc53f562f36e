"""Local discrete convolution with the DGF (paper sec. 2, eq.
discreteConvolution; sec. 4.1 step 1; Hockney's method in appendix A.2).

Everything here works in h = 1 units: the result is
    out[x] = sum_j G1[x - j] q[j]
and the caller multiplies by h^2 (because G^h = G1 / h and the discrete
convolution carries h^3).

The source q is given on a box [0, S0-1] x [0, S1-1] x [0, S2-1] (relative
coordinates) and the output is wanted on [olo, ohi] (relative coordinates,
closed).  G1 is the table returned by oracle.dgf.dgf, centre index Z.
"""
import numpy as np
import scipy.fft as sfft


def _kernel_slice(G1, Z, lo, hi):
    """G1 restricted to offsets lo..hi (closed, per axis)."""
    if np.any(np.asarray(lo) < -Z) or np.any(np.asarray(hi) > Z):
        raise ValueError("DGF table too small for the requested offsets")
    return G1[Z + lo[0]:Z + hi[0] + 1, Z + lo[1]:Z + hi[1] + 1, Z + lo[2]:Z + hi[2] + 1]


def conv_direct(G1, Z, q, olo, ohi):
    """The literal sum out[x] = sum_j G1[x-j] q[j], accumulated one source
    node at a time.  Slow; meant for small cases and sampled checks."""
    olo = np.asarray(olo)
    ohi = np.asarray(ohi)
    shape = tuple(ohi - olo + 1)
    out = np.zeros(shape)
    for j in zip(*np.nonzero(q)):
        j = np.asarray(j)
        out += q[tuple(j)] * _kernel_slice(G1, Z, olo - j, ohi - j)
    return out


def conv_direct_at(G1, Z, q, pts):
    """out[x] for a list of points x (shape (m, 3)), by the literal sum."""
    pts = np.asarray(pts)
    S = np.array(q.shape)
    res = np.empty(len(pts))
    for t, x in enumerate(pts):
        k = _kernel_slice(G1, Z, x - S + 1, x)
        # k[a] = G1[x - (S-1) + a] = G1[x - j] with j = S-1-a
        res[t] = np.sum(k[::-1, ::-1, ::-1] * q)
    return res


def conv_hockney(G1, Z, q, olo, ohi, M=None, kernel_cache=None):
    """Hockney's method (appendix A.2), per axis: the source occupies
    [0, b] (b = S-1), the output [olo, ohi]; shift the output to [0, n']
    with n' = ohi - olo and the source to [-olo - ..].  Concretely, with
    sigma = olo the kernel offsets x - j run over [olo - b, ohi]; the paper
    periodises kernel and source on an interval of length n' + b' + 1 with
    b' >= b and evaluates the periodic convolution by the DFT.  The kernel
    is placed on the offsets [ohi - (M-1), ohi] (the interval [-b', n']
    shifted by olo), which contains the needed offsets [olo - b, ohi].
    """
    olo = np.asarray(olo)
    ohi = np.asarray(ohi)
    S = np.array(q.shape)
    npr = ohi - olo                        # n' per axis
    Mmin = npr + S                         # n' + b + 1 with b = S - 1
    if M is None:
        M = [sfft.next_fast_len(int(m), real=True) for m in Mmin]
    M = np.broadcast_to(np.asarray(M), (3,)).copy()
    if np.any(M < Mmin):
        raise ValueError("torus too small for an exact convolution")
    # kernel on offsets t in [ohi - M + 1, ohi]; torus slot of offset t is
    # (t - olo) mod M, so that output x sits at slot x - olo in [0, n'].
    key = (id(G1), tuple(olo), tuple(ohi), tuple(M))
    if kernel_cache is not None and key in kernel_cache:
        khat = kernel_cache[key]
    else:
        klo = ohi - M + 1
        kern = _kernel_slice(G1, Z, klo, ohi)
        kt = np.zeros(tuple(M))
        idx = [np.mod(np.arange(klo[d], ohi[d] + 1) - olo[d], M[d]) for d in range(3)]
        kt[np.ix_(*idx)] = kern
        khat = sfft.rfftn(kt)
        if kernel_cache is not None:
            kernel_cache[key] = khat
    # source j sits at slot j (its offset contribution: out slot x - olo
    # receives kern at slot (x - olo - j) mod M = offset x - j)
    st = np.zeros(tuple(M))
    st[:S[0], :S[1], :S[2]] = q
    prod = khat * sfft.rfftn(st)
    full = sfft.irfftn(prod, s=tuple(M))
    return full[:npr[0] + 1, :npr[1] + 1, :npr[2] + 1].copy()
