"""The paper's own error tables for the smooth charge (sec. 7.1), reproduced
by the float64 GPU path at N = 256 (MI355X only).

Loose pin: the interpolation operator I^H is a reading of the paper (it
defers the operator to earlier work), so exact agreement is not expected;
each error must be within a factor 4 of the printed value, and the trends the
paper reports must hold (tests/golden/smooth_charge_two_level_errors.txt).
The L19 rows with the Legendre far field at P = 4 (beta > alpha), whose
error is not dominated by the interpolation, must agree within 20 %.  The
rows cover every N = 256 entry of Tables 1-7 that the build runs (alpha <= 3):
L19 and L27, P = 1, 4, 5, 6 and 9 (P >= 5 with the full Boole Gram matrix).

Tables 5 and 6 (L27 with alpha = 1.5, whose Omega_alpha has an 8-cell
margin at n = 32) are where the reading of I^H shows: the paper states a
stencil radius b = 3, whose stencil under this reading (2b + 2 coplanar
coarse nodes per axis around the node's coarse cell, reaching about 15 fine
cells) extends past the margin, and the errors come out 6-23 times the
printed ones; with radius 2 (about 11 cells) the P = 4 rows agree within 5 %.
At alpha = 1.75 (Table 7, a 12-cell margin) radius 3 agrees within 30 %.  So
those two tables run at both radii: the radius-2 far-field rows must agree
within 20 % and the radius-3 errors are reported."""
import os

import numpy as np
import pytest

import mlc_inputs as mi
from paper_1702_08111_amd import mlc as gm

from gpu_common import gpu_solve

pytestmark = pytest.mark.gpu

N, n = 256, 32


def _rows():
    path = os.path.join(os.path.dirname(__file__), "golden", "smooth_charge_two_level_errors.txt")
    out = []
    for ln in open(path):
        if ln.strip() and not ln.startswith("#"):
            t, Q, a, b, P, e = ln.split()
            out.append((t, int(Q), float(a), float(b), int(P), float(e)))
    return out


@pytest.fixture(scope="module")
def errors():
    f = mi.smooth_charge(N)
    exact = mi.smooth_potential(N)
    scale = np.abs(exact).max()
    out = {}
    for t, Q, a, b, P, paper in _rows():
        g = gpu_solve(gm.problem(N, n, a, b, P, Q, conv="fp64"), f, keep=False)
        out[(t, Q, a, b, P)] = (float(np.abs(g["phi"] - exact).max() / scale), paper)
        print(t, Q, a, b, P, f"{out[(t, Q, a, b, P)][0]:.3e} (paper {paper:.3e})", flush=True)
        if t in NARROW_STENCIL:
            g = gpu_solve(gm.problem(N, n, a, b, P, Q, b=2, conv="fp64"), f, keep=False)
            out[(t + "_b2", Q, a, b, P)] = (float(np.abs(g["phi"] - exact).max() / scale), paper)
            print(t, "interpolation radius 2:", f"{out[(t + '_b2', Q, a, b, P)][0]:.3e}", flush=True)
    return out


# the tables whose stated radius-3 stencil reaches past Omega_alpha under the
# reading of I^H (module docstring)
NARROW_STENCIL = ("table5", "table6")


def test_same_order_as_paper(errors):
    for key, (e, paper) in errors.items():
        if key[0] in NARROW_STENCIL:
            continue
        assert paper / 4 < e < paper * 4, (key, e, paper)


def test_narrow_stencil_tables(errors):
    """Tables 5-6: radius-2 P = 4 rows within 20 % of the paper, and the
    stated radius 3 worse than radius 2 under this reading."""
    for t in NARROW_STENCIL:
        keys = [k for k in errors if k[0] == t]
        assert keys
        for k in keys:
            e3, paper = errors[k]
            e2 = errors[(t + "_b2",) + k[1:]][0]
            assert e2 < e3, (k, e2, e3)
            if k[4] == 4:
                assert abs(e2 / paper - 1.0) < 0.2, (k, e2, paper)


def test_far_field_rows_within_20_percent(errors):
    rows = [(k, v) for k, v in errors.items() if k[1] == 4 and k[4] == 4 and k[3] > k[2] and "_b2" not in k[0]]
    assert rows
    for key, (e, paper) in rows:
        assert abs(e / paper - 1.0) < 0.2, (key, e, paper)


def test_paper_trends(errors):
    # doubling beta without the far field cuts the barrier error >= 16x (L19)
    assert errors[("table1", 4, 1.5, 1.5, 4)][0] / errors[("table1", 4, 3.0, 3.0, 4)][0] > 10
    # the Legendre far field (P = 4) beats P = 1 at equal radii (Tables 2-3)
    for t, b in (("table2", 3.0), ("table3", 6.0)):
        assert errors[(t, 4, 1.5, b, 4)][0] < errors[(t, 4, 1.5, b, 1)][0]
    # and beats the far-field-free method at the same inner radius
    assert errors[("table2", 4, 1.5, 3.0, 4)][0] < errors[("table1", 4, 1.5, 1.5, 4)][0]
    # L27, alpha 1.75, beta 3.25: a high Legendre degree is needed at N = 256
    # (Table 7): P = 9 < P = 6 < P = 4
    t7 = [errors[("table7", 6, 1.75, 3.25, P)][0] for P in (4, 6, 9)]
    assert t7[0] > t7[1] > t7[2], t7
