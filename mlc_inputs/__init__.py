"""Seeded synthetic charges on the unit cube and their closed-form potentials.

Shared by the tests, the benchmark and the smoke check; it holds none of the
solver's arithmetic (no stencils, Green's functions, transforms or moments),
only charge densities sampled on nodes and the exact continuous potentials
they induce under Delta phi = f with phi -> -q/(4 pi |x|).

Charges
  bump      f = w (1 - rho^2)^4 for rho = |x - c| / R < 1, else 0.
            phi = w R^2 psi(rho),
            psi = rho^2/6 - rho^4/5 + rho^6/7 - rho^8/18 + rho^10/110 - 1/10
                  (rho < 1),   -128 / (3465 rho)  (rho >= 1).
  smooth    the paper's smooth test charge (sec. 7.1): f = (r - r^2)^4 for
            r = |x - x0| / Ro < 1, Ro = 1/4, x0 = (1/2, 1/2, 1/2), with the
            potential printed there.
  oscillatory  the three oscillatory charges of sec. 7.2:
            f = Ro^-3 (r - r^2)^2 sin^2(gamma r / 2), Ro = 1/20,
            gamma = 28 pi, centres printed there, with the printed potential.

Workloads (seeded with numpy's PCG64; per bump: centre (3 uniforms),
radius, weight, in that order):
  one_bump      config 'plain FP64, 32^3': w = 1, R = 0.35, centre (1/2)^3
  bumps(k, ...) k bumps, centres U[lo, hi]^3, radii U(r0, r1), weights U(-1, 1)
  batch_problems  uneven batch: per problem N ~ U{sizes}, then the bump count
                U{1..4}, then its bumps, all from one stream
  serving_requests  request mix: per request N, n, Q, bump count, bumps;
                arrival gaps Exp(1/rate) from a second stream
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Bump:
    centre: tuple
    radius: float
    weight: float


def _rho(N, c, R):
    ax = np.arange(N + 1) / N
    d0 = (ax - c[0])[:, None, None]
    d1 = (ax - c[1])[None, :, None]
    d2 = (ax - c[2])[None, None, :]
    return np.sqrt(d0 * d0 + d1 * d1 + d2 * d2) / R


def bump_charge(N, bumps):
    """Sum of bump charges sampled on the (N+1)^3 nodes g/N of [0, 1]^3
    (each bump evaluated on the nodes of its bounding box only; it is zero
    elsewhere)."""
    f = np.zeros((N + 1,) * 3)
    ax = np.arange(N + 1) / N
    for bp in bumps:
        c, R = bp.centre, bp.radius
        box = []
        for d in range(3):
            lo = max(int(np.floor((c[d] - R) * N)) - 1, 0)
            hi = min(int(np.ceil((c[d] + R) * N)) + 1, N)
            box.append(slice(lo, hi + 1))
        d0 = (ax[box[0]] - c[0])[:, None, None]
        d1 = (ax[box[1]] - c[1])[None, :, None]
        d2 = (ax[box[2]] - c[2])[None, None, :]
        r = np.sqrt(d0 * d0 + d1 * d1 + d2 * d2) / R
        f[tuple(box)] += bp.weight * np.where(r < 1.0, (1.0 - r * r) ** 4, 0.0)
    return f


def _psi_bump(r):
    r2 = r * r
    inside = r2 / 6 - r2 ** 2 / 5 + r2 ** 3 / 7 - r2 ** 4 / 18 + r2 ** 5 / 110 - 0.1
    rs = np.where(r > 0, r, 1.0)
    outside = -128.0 / (3465.0 * rs)
    return np.where(r < 1.0, inside, outside)


def bump_potential(N, bumps):
    """Closed-form potential of bump_charge on the same nodes."""
    phi = np.zeros((N + 1,) * 3)
    for bp in bumps:
        r = _rho(N, bp.centre, bp.radius)
        phi += bp.weight * bp.radius ** 2 * _psi_bump(r)
    return phi


def bump_potential_at(x, bumps):
    """Closed-form potential at arbitrary points x (shape (m, 3))."""
    x = np.asarray(x, dtype=np.float64)
    phi = np.zeros(len(x))
    for bp in bumps:
        r = np.linalg.norm(x - np.asarray(bp.centre), axis=1) / bp.radius
        phi += bp.weight * bp.radius ** 2 * _psi_bump(r)
    return phi


SMOOTH_RO = 0.25


def smooth_charge(N):
    """The paper's smooth charge (sec. 7.1) on the nodes of [0, 1]^3."""
    r = _rho(N, (0.5, 0.5, 0.5), SMOOTH_RO)
    return np.where(r < 1.0, (r - r * r) ** 4, 0.0)


def smooth_potential(N):
    """The closed-form potential printed with the smooth charge (sec. 7.1)."""
    r = _rho(N, (0.5, 0.5, 0.5), SMOOTH_RO)
    inside = (r ** 6 / 42 - r ** 7 / 14 + r ** 8 / 12 - 2 * r ** 9 / 45 + r ** 10 / 110 - 1.0 / 1260)
    rs = np.where(r > 0, r, 1.0)
    outside = -1.0 / (2310.0 * rs)
    return SMOOTH_RO ** 2 * np.where(r < 1.0, inside, outside)


# A smoother radial charge for order-of-accuracy checks beyond fourth order:
# f = (1 - rho^2)^k inside the ball rho = |x - c| / R < 1 (C^(k-1) across its
# surface), with the potential of Delta phi = f that decays at infinity,
#   phi(r) = -(1/r) int_0^min(r,R) f s^2 ds - int_min(r,R)^R f s ds,
# integrated exactly as polynomials in s.
def _poly_profile_integrals(k):
    from numpy.polynomial import polynomial as npoly
    base = npoly.polypow([1.0, 0.0, -1.0], k)          # (1 - u^2)^k in u = s / R
    m2 = npoly.polyint(npoly.polymul(base, [0.0, 0.0, 1.0]))   # int_0^u t^2 f dt
    m1 = npoly.polyint(npoly.polymul(base, [0.0, 1.0]))        # int_0^u t f dt
    return m2, m1


def poly_charge(N, k=10, centre=(0.5, 0.5, 0.5), R=0.3):
    r = _rho(N, centre, R)
    return np.where(r < 1.0, (1.0 - r * r) ** k, 0.0)


def poly_potential(N, k=10, centre=(0.5, 0.5, 0.5), R=0.3):
    from numpy.polynomial import polynomial as npoly
    m2, m1 = _poly_profile_integrals(k)
    u = np.minimum(_rho(N, centre, R), 1.0)
    r = _rho(N, centre, R)
    rs = np.where(r > 0, r, 1.0)
    inner = np.where(r > 0, npoly.polyval(u, m2) / rs, 0.0)     # (1/u) int_0^u t^2 f dt (in units of R)
    outer = npoly.polyval(1.0, m1) - npoly.polyval(u, m1)        # int_u^1 t f dt
    return -R * R * (inner + outer)


# The oscillatory three-charge test of sec. 7.2: each charge is supported in
# a ball of radius OSC_RO, with gamma = 4 mu pi, mu = 7.
OSC_RO = 0.05
OSC_GAMMA = 28.0 * np.pi
OSC_CENTRES = ((3 / 16, 7 / 16, 13 / 16), (7 / 16, 13 / 16, 3 / 16), (13 / 16, 3 / 16, 7 / 16))


def _osc_profile(r, g=OSC_GAMMA):
    """(r - r^2)^2 sin^2(g r / 2) inside the unit ball, 0 outside."""
    return np.where(r < 1.0, (r - r * r) ** 2 * np.sin(0.5 * g * r) ** 2, 0.0)


def _osc_psi(r, g=OSC_GAMMA, xp=np):
    """The dimensionless potential of one oscillatory charge (sec. 7.2): the
    potential is psi(|x - x_o| / Ro) / Ro.  xp: the array module (numpy, or
    torch for device arrays)."""
    r = xp.asarray(r, dtype=xp.float64)
    rs = xp.where(r > 0, r, 1.0)
    c, sn = xp.cos(g * rs), xp.sin(g * rs)
    inside = (rs ** 6 / 84 - rs ** 5 / 30 + rs ** 4 / 40 + 60 / g ** 6 - 9 / g ** 4 - 1 / 120 + 120 / (g ** 6 * rs)
              + (-120 / (g ** 6 * rs) - 9 / g ** 4 + 300 / g ** 6 + 36 * rs / g ** 4 + rs ** 2 / (2 * g ** 2)
                 - 30 * rs ** 2 / g ** 4 - rs ** 3 / g ** 2 + rs ** 4 / (2 * g ** 2)) * c
              + (12 / (g ** 5 * rs) - 360 / (g ** 7 * rs) - 96 / g ** 5 + 120 * rs / g ** 5 - 3 * rs / g ** 3
                 + 8 * rs ** 2 / g ** 3 - 5 * rs ** 3 / g ** 3) * sn)
    outside = (-1.0 / 210 - 12 / g ** 4 + 360 / g ** 6) / rs
    at0 = -1.0 / 120 - 6 / g ** 4
    return xp.where(r == 0, at0, xp.where(r < 1.0, inside, outside))


def oscillatory_charge(N):
    """The sum of the three oscillatory charges of sec. 7.2 on the (N+1)^3
    nodes of [0, 1]^3: f = Ro^-3 (r - r^2)^2 sin^2(gamma r / 2), r = |x - c| / Ro."""
    f = np.zeros((N + 1,) * 3)
    ax = np.arange(N + 1) / N
    for c in OSC_CENTRES:
        box = []
        for d in range(3):
            lo = max(int(np.floor((c[d] - OSC_RO) * N)) - 1, 0)
            hi = min(int(np.ceil((c[d] + OSC_RO) * N)) + 1, N)
            box.append(slice(lo, hi + 1))
        d0 = (ax[box[0]] - c[0])[:, None, None]
        d1 = (ax[box[1]] - c[1])[None, :, None]
        d2 = (ax[box[2]] - c[2])[None, None, :]
        r = np.sqrt(d0 * d0 + d1 * d1 + d2 * d2) / OSC_RO
        f[tuple(box)] += _osc_profile(r) / OSC_RO ** 3
    return f


def oscillatory_potential(N):
    """The closed-form potential of oscillatory_charge on the same nodes."""
    phi = np.zeros((N + 1,) * 3)
    for c in OSC_CENTRES:
        phi += _osc_psi(_rho(N, c, OSC_RO)) / OSC_RO
    return phi


# Charges as sums of radial terms (centre, radius, weight, param, profile):
# f(x) = weight * profile(|x - centre| / radius) inside the ball, 0 outside.
PROFILE_BUMP, PROFILE_SMOOTH, PROFILE_OSCILLATORY = 0, 1, 2


def _profile(kind, r, param):
    if kind == PROFILE_BUMP:
        v = (1.0 - r * r) ** 4
    elif kind == PROFILE_SMOOTH:
        v = (r - r * r) ** 4
    else:
        v = (r - r * r) ** 2 * np.sin(0.5 * param * r) ** 2
    return np.where(r < 1.0, v, 0.0)


def radial_charge_at(x0, x1, x2, terms):
    """f at points with coordinates x0, x1, x2 (arrays that broadcast)."""
    f = 0.0
    for c, R, w, param, kind in terms:
        r = np.sqrt((x0 - c[0]) ** 2 + (x1 - c[1]) ** 2 + (x2 - c[2]) ** 2) / R
        f = f + w * _profile(kind, r, param)
    return f


def radial_charge_nodes(N, terms):
    """f on the (N+1)^3 nodes g / N of [0, 1]^3."""
    ax = np.arange(N + 1) / N
    return np.asarray(radial_charge_at(ax[:, None, None], ax[None, :, None], ax[None, None, :], terms),
                      dtype=np.float64) * np.ones((N + 1,) * 3)


def bump_terms(bumps):
    return [(b.centre, b.radius, b.weight, 0.0, PROFILE_BUMP) for b in bumps]


def smooth_terms():
    """The smooth charge of sec. 7.1 as one radial term."""
    return [((0.5, 0.5, 0.5), SMOOTH_RO, 1.0, 0.0, PROFILE_SMOOTH)]


def oscillatory_terms():
    """The three oscillatory charges of sec. 7.2 as radial terms."""
    return [(c, OSC_RO, OSC_RO ** -3, OSC_GAMMA, PROFILE_OSCILLATORY) for c in OSC_CENTRES]


def one_bump():
    return [Bump((0.5, 0.5, 0.5), 0.35, 1.0)]


def _draw_bumps(rng, k, radius, centre):
    out = []
    for _ in range(k):
        c = tuple(float(v) for v in rng.uniform(centre[0], centre[1], size=3))
        R = float(rng.uniform(radius[0], radius[1]))
        w = float(rng.uniform(-1.0, 1.0))
        out.append(Bump(c, R, w))
    return out


def bumps(k, seed, radius=(0.1, 0.2), centre=(0.3, 0.7)):
    """k seeded bumps; centres U[centre]^3, radii U(radius), weights U(-1, 1)."""
    return _draw_bumps(np.random.Generator(np.random.PCG64(seed)), k, radius, centre)


BATCH_SIZES = (32, 64, 96, 128, 192)


def batch_problems(count=64, seed=104, sizes=BATCH_SIZES, radius=(0.1, 0.2), centre=(0.3, 0.7)):
    """Uneven batch: [(N, bumps)], N ~ U{sizes}, 1-4 bumps each."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        N = int(sizes[int(rng.integers(0, len(sizes)))])
        k = int(rng.integers(1, 5))
        out.append((N, _draw_bumps(rng, k, radius, centre)))
    return out


SERVING_SIZES = (64, 128, 192, 256)


def serving_requests(count, rate, seed=105, sizes=SERVING_SIZES, patches=(16, 32), orders=(4, 6)):
    """Request stream: [(t_arrival, N, n, Q, bumps)] with Poisson arrivals at
    `rate` per second (gaps from a second stream seeded seed + 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = np.random.Generator(np.random.PCG64(seed + 1)).exponential(1.0 / rate, size=count)
    out = []
    t = 0.0
    for i in range(count):
        N = int(sizes[int(rng.integers(0, len(sizes)))])
        n = int(patches[int(rng.integers(0, len(patches)))])
        Q = int(orders[int(rng.integers(0, len(orders)))])
        k = int(rng.integers(1, 5))
        t += float(gaps[i])
        out.append((t, N, n, Q, _draw_bumps(rng, k, (0.1, 0.2), (0.3, 0.7))))
    return out


# the named workloads: (N, n, Q, bumps)
WORKLOADS = {
    "fp64_32": dict(N=32, n=8, Q=4, bumps=lambda: one_bump()),
    "fp32_128": dict(N=128, n=16, Q=4, bumps=lambda: bumps(3, 102)),
    "fp32_256_q6": dict(N=256, n=32, Q=6, bumps=lambda: bumps(8, 103, radius=(0.05, 0.15))),
    "fp32_256_q4": dict(N=256, n=32, Q=4, bumps=lambda: bumps(8, 103, radius=(0.05, 0.15))),
}


def workload(name):
    """(N, n, Q, bumps) of a named workload."""
    w = WORKLOADS[name]
    return w["N"], w["n"], w["Q"], w["bumps"]()
