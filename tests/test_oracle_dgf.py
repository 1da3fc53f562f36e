"""Pins of the discrete Green's function (paper sec. 2 eq. dgf, appendix A.1)."""
import numpy as np
import pytest

from oracle.dgf import dgf, dgf_cached
from oracle.stencils import apply_laplacian

# Watson's integral for the simple cubic lattice: the lattice Green's
# function of the 7-point Laplacian at the origin is -W/6 with
# W = 1.516386059151978... (G. N. Watson, 1939), so G(0) = -0.25273100985866.
WATSON_G0 = -1.5163860591519780 / 6.0


@pytest.mark.parametrize("Q", [4, 6])
def test_dgf_is_inverse_of_stencil(Q):
    """L G1 = delta_0 on the interior of the table."""
    Z = 24
    G1 = dgf(Q, Z)
    r = apply_laplacian(G1, Q)
    r[Z - 1, Z - 1, Z - 1] -= 1.0
    assert np.abs(r).max() < 1e-13


@pytest.mark.parametrize("Q", [4, 6])
def test_dgf_symmetry(Q):
    """48-fold symmetry of the cube (reflections and axis permutations)."""
    G1 = dgf(Q, 16)
    for perm in [(1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0)]:
        assert np.abs(G1 - np.transpose(G1, perm)).max() < 1e-15
    for ax in range(3):
        assert np.abs(G1 - np.flip(G1, ax)).max() < 1e-15


def test_watson_value_7point():
    """The same solver applied to the 7-point Laplacian reproduces Watson's
    value of the lattice Green's function at the origin."""
    G = dgf(2, 64)
    assert abs(G[64, 64, 64] - WATSON_G0) < 2e-6


@pytest.mark.parametrize("Q", [4, 6])
def test_dgf_far_field(Q, dgf64_q4, dgf64_q6):
    """G1[g] -> -1/(4 pi |g|) (sec. 2): relative gap decays with |g|."""
    G1 = dgf64_q4 if Q == 4 else dgf64_q6
    Z = 64
    gaps = []
    for r in (8, 16, 32):
        for g in [(r, 0, 0), (r, r, 0), (r, r, r), (r, r // 2, 3)]:
            exact = -1.0 / (4 * np.pi * np.linalg.norm(g))
            gaps.append((r, abs(G1[Z + g[0], Z + g[1], Z + g[2]] / exact - 1.0)))
    by_r = {r: max(v for rr, v in gaps if rr == r) for r in (8, 16, 32)}
    assert by_r[8] < 1e-3
    assert by_r[32] < by_r[16] < by_r[8]


@pytest.mark.parametrize("Q", [4, 6])
def test_dgf_converges_with_table_size(Q):
    """The boundary-condition error decays like (zeta Z)^-4 (appendix A.1):
    doubling Z shrinks the change on [-8, 8]^3 by roughly 16."""
    Gs = {Z: dgf(Q, Z) for Z in (16, 32, 64)}
    c = 8

    def core(Z):
        return Gs[Z][Z - c:Z + c + 1, Z - c:Z + c + 1, Z - c:Z + c + 1]

    d1 = np.abs(core(16) - core(32)).max()
    d2 = np.abs(core(32) - core(64)).max()
    assert d2 < d1 / 8
    assert d2 < 1e-7


def test_paper_ten_digits_claim():
    """Z = 128 and zeta = 2 give at least ten digits (appendix A.1):
    the Z = 64 and Z = 128 tables agree to ~1e-10 relative near the origin."""
    a = dgf_cached(4, 64)
    b = dgf_cached(4, 128)
    c = 16
    da = a[64 - c:64 + c + 1, 64 - c:64 + c + 1, 64 - c:64 + c + 1]
    db = b[128 - c:128 + c + 1, 128 - c:128 + c + 1, 128 - c:128 + c + 1]
    # the Z=64 table carries the (larger) error; Z=128 is ~16x better still
    assert np.abs(da - db).max() / np.abs(db).max() < 2e-9
