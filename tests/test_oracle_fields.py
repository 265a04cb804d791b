"""Pins of the coefficient fields (Sections 2 and 4): the manufactured
solution of eq. 46 and its derivatives against symbolic differentiation, and
the layout of the Section 4 workload."""
import math

import numpy as np
import pytest

import workloads
from oracle import fields, geometry


def _symbolic_jet():
    sympy = pytest.importorskip("sympy")
    x, y = sympy.symbols("x y", real=True)
    u = (3 + sympy.Rational(1, 3) * sympy.sin(sympy.sqrt(1 + x ** 2 / 100 + y ** 2 / 50))
         + sympy.Rational(1, 3) * sympy.tanh(sympy.sin(3 * x / 25 + y / 20)
                                             + sympy.sin(x / 20 - 3 * y / 25)))
    parts = [u, sympy.diff(u, x), sympy.diff(u, y), sympy.diff(u, x, 2), sympy.diff(u, x, y),
             sympy.diff(u, y, 2)]
    return [sympy.lambdify((x, y), p, "numpy") for p in parts]


def test_eq46_value_at_the_origin():
    # rho = 1 and s = 0 at the origin: u = 3 + sin(1) / 3
    assert fields.value({"kind": "eq46"}, 0.0, 0.0) == pytest.approx(3.0 + math.sin(1.0) / 3.0, abs=1e-15)


def test_eq46_jet_matches_symbolic_derivatives():
    ref = _symbolic_jet()
    rng = np.random.default_rng(46)
    x = rng.uniform(-750.0, 750.0, size=200)
    y = rng.uniform(-750.0, 750.0, size=200)
    got = fields.jet({"kind": "eq46"}, x, y)
    for k in range(6):
        want = np.broadcast_to(ref[k](x, y), x.shape)
        scale = max(1.0, float(np.max(np.abs(want))))
        assert np.max(np.abs(got[k] - want)) <= 1e-13 * scale, k


def test_eq46_derived_source_is_minus_the_laplacian():
    # Poisson with a_xx = a_yy = 2: f = -(u_xx + u_yy)
    ref = _symbolic_jet()
    cfg = workloads.paper_poisson()
    prob = cfg["problem"]
    rng = np.random.default_rng(7)
    x = rng.uniform(-50.0, 50.0, size=50)
    y = rng.uniform(-50.0, 50.0, size=50)
    f = fields.value(prob["f"], x, y, prob)
    lap = ref[3](x, y) + ref[5](x, y)
    assert np.max(np.abs(f + lap)) <= 1e-15 * 50


def test_section4_workload_layout():
    # 100 circles on a lattice of spacing 10 in [-50, 50]^2, radii in
    # [8.55, 9.43], 44 knots and 44 x 22 nodes; the outer ring of 36 circles
    # crosses the boundary
    cfg = workloads.paper_poisson()
    cov = cfg["cover"]
    assert len(cov["radii"]) == 100
    assert np.all((cov["radii"] >= 8.55) & (cov["radii"] <= 9.43))
    xs = np.unique(cov["centres"][:, 0])
    assert np.allclose(np.diff(xs), 10.0) and xs[0] == -45.0
    assert np.all(cov["M"] == 44) and np.all(cov["Ntheta"] == 44) and np.all(cov["Nr"] == 22)
    cv = geometry.build_cover(cfg["problem"]["domain"], cov)
    assert int(np.sum(cv.floating)) == 64
