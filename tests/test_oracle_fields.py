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


def _symbolic_sinsum(fd):
    """The SINSUM field as a sympy expression of (x, y), with its jet."""
    sympy = pytest.importorskip("sympy")
    x, y = sympy.symbols("x y", real=True)
    u = sympy.Float(fd["base"])
    for a, kx, ky, p in zip(fd["amp"], fd["kx"], fd["ky"], fd["phase"]):
        u = u + sympy.Float(a) * sympy.sin(2 * sympy.pi * (sympy.Float(kx) * x + sympy.Float(ky) * y)
                                           + sympy.Float(p))
    parts = [u, sympy.diff(u, x), sympy.diff(u, y), sympy.diff(u, x, 2), sympy.diff(u, x, y),
             sympy.diff(u, y, 2)]
    return [sympy.lambdify((x, y), q, "numpy") for q in parts]


@pytest.mark.parametrize("name", ["config2", "small_variable"])
def test_sinsum_jet_matches_symbolic_derivatives(name):
    # the manufactured solutions of the variable-coefficient workloads (eq. 1's
    # u): the hand-derived jet against sympy's differentiation of the same sum
    cfg = workloads.config2() if name == "config2" else workloads.small_variable()
    ufd = cfg["problem"]["u_exact"]
    ref = _symbolic_sinsum(ufd)
    rng = np.random.default_rng(12)
    x = rng.uniform(-0.2, 1.2, size=300)
    y = rng.uniform(-0.2, 1.2, size=300)
    got = fields.jet(ufd, x, y)
    for k in range(6):
        want = np.broadcast_to(ref[k](x, y), x.shape)
        scale = max(1.0, float(np.max(np.abs(want))))
        assert np.max(np.abs(got[k] - want)) <= 1e-12 * scale, k


@pytest.mark.parametrize("name", ["config2", "small_variable"])
def test_derived_source_matches_finite_differences_of_the_operator(name):
    # f = -(L u + c u) of eq. 1 with L = a_xx/2 d_xx + a_xy d_xy + a_yy/2 d_yy
    # + b . grad, the derivatives of u taken by fourth-order central
    # differences of its values (not its jet); small_variable has a_xy != 0
    cfg = workloads.config2() if name == "config2" else workloads.small_variable()
    prob = cfg["problem"]
    ufd = prob["u_exact"]
    rng = np.random.default_rng(13)
    x = rng.uniform(0.0, 1.0, size=200)
    y = rng.uniform(0.0, 1.0, size=200)
    d = 1e-3

    def U(dx, dy):
        return fields.value(ufd, x + dx * d, y + dy * d)

    w = {-2: 1.0 / 12, -1: -2.0 / 3, 1: 2.0 / 3, 2: -1.0 / 12}
    w2 = {-2: -1.0 / 12, -1: 4.0 / 3, 0: -5.0 / 2, 1: 4.0 / 3, 2: -1.0 / 12}
    ux = sum(c * U(s, 0) for s, c in w.items()) / d
    uy = sum(c * U(0, s) for s, c in w.items()) / d
    uxx = sum(c * U(s, 0) for s, c in w2.items()) / d ** 2
    uyy = sum(c * U(0, s) for s, c in w2.items()) / d ** 2
    uxy = sum(ci * cj * U(si, sj) for si, ci in w.items() for sj, cj in w.items()) / d ** 2
    co = {k: fields.value(prob[k], x, y) for k in ("axx", "axy", "ayy", "bx", "by", "c")}
    f_fd = -(0.5 * co["axx"] * uxx + co["axy"] * uxy + 0.5 * co["ayy"] * uyy + co["bx"] * ux
             + co["by"] * uy + co["c"] * U(0, 0))
    f = fields.value(prob["f"], x, y, prob)
    assert np.max(np.abs(f - f_fd)) <= 1e-6 * max(1.0, float(np.max(np.abs(f))))


def test_sigma_is_the_cholesky_factor_of_a():
    # eq. 3: sigma sigma^T = [[a_xx, a_xy], [a_xy, a_yy]], sigma lower triangular
    # with a positive diagonal, including a_xy != 0
    rng = np.random.default_rng(14)
    L = np.tril(rng.uniform(-1.0, 1.0, size=(50, 2, 2)))
    L[:, 0, 0] = np.abs(L[:, 0, 0]) + 0.1
    L[:, 1, 1] = np.abs(L[:, 1, 1]) + 0.1
    A = L @ np.transpose(L, (0, 2, 1))
    s11, s21, s22 = fields.sigma(A[:, 0, 0], A[:, 0, 1], A[:, 1, 1])
    assert np.max(np.abs(s11 - L[:, 0, 0])) < 1e-14
    assert np.max(np.abs(s21 - L[:, 1, 0])) < 1e-14
    assert np.max(np.abs(s22 - L[:, 1, 1])) < 1e-14
