"""Pins for the oracle's polar collocation (Section 3.3) and floating rows
(Section 2.4, eqs. 31-35)."""
import math

import numpy as np
import pytest

import workloads
from oracle import cardinal, fields, geometry, spectral


def test_chebyshev_diff_matches_textbook_closed_form():
    # Chebyshev differentiation matrix in closed form (Trefethen, Spectral
    # Methods in MATLAB, ch. 6) against the oracle's Lagrange-basis definition.
    N = 13
    x = spectral.cheb_points(N)
    c = np.ones(N + 1)
    c[0] = c[N] = 2.0
    D = np.zeros((N + 1, N + 1))
    for i in range(N + 1):
        for j in range(N + 1):
            if i != j:
                D[i, j] = (c[i] / c[j]) * (-1) ** (i + j) / (x[i] - x[j])
    for j in range(1, N):
        D[j, j] = -x[j] / (2 * (1 - x[j] ** 2))
    D[0, 0] = (2 * N * N + 1) / 6.0
    D[N, N] = -D[0, 0]
    assert np.max(np.abs(spectral.lagrange_diff(x) - D)) < 1e-11


def _poly(rng, deg):
    coef = rng.standard_normal((deg + 1, deg + 1))
    coef[np.add.outer(np.arange(deg + 1), np.arange(deg + 1)) > deg] = 0.0

    def jet(x, y):
        u = ux = uy = uxx = uxy = uyy = 0.0
        for a in range(deg + 1):
            for b in range(deg + 1 - a):
                cf = coef[a, b]
                u = u + cf * x ** a * y ** b
                if a >= 1:
                    ux = ux + cf * a * x ** (a - 1) * y ** b
                if b >= 1:
                    uy = uy + cf * b * x ** a * y ** (b - 1)
                if a >= 2:
                    uxx = uxx + cf * a * (a - 1) * x ** (a - 2) * y ** b
                if b >= 2:
                    uyy = uyy + cf * b * (b - 1) * x ** a * y ** (b - 2)
                if a >= 1 and b >= 1:
                    uxy = uxy + cf * a * b * x ** (a - 1) * y ** (b - 1)
        return u, ux, uy, uxx, uxy, uyy
    return jet


def _ring_xy(grid, cx, cy, r):
    return cx + r * np.cos(grid.theta), cy + r * np.sin(grid.theta)


def test_polar_operators_differentiate_polynomials_exactly():
    grid = spectral.local_grid(7, 16)
    cx, cy, r = 0.3, -0.2, 0.7
    jet = _poly(np.random.default_rng(4), 6)
    xi, yi = grid.node_xy(cx, cy, r)
    xb, yb = _ring_xy(grid, cx, cy, r)
    vals = np.concatenate([jet(xi, yi)[0], jet(xb, yb)[0]])
    u, ux, uy, uxx, uxy, uyy = jet(xi, yi)
    ops = grid.physical_ops(r)
    scale = np.max(np.abs(uxx)) + 1
    for name, ref in (("x", ux), ("y", uy), ("xx", uxx), ("xy", uxy), ("yy", uyy)):
        assert np.max(np.abs(ops[name] @ vals - ref)) < 1e-10 * scale, name


def test_polynomial_reproduction_with_arbitrary_coefficients():
    # Collocation is exact on its own space: with f := -(L u_p + c u_p) at the
    # nodes and ring data u_p, the discrete solution is u_p at the nodes.
    grid = spectral.local_grid(6, 16)
    cx, cy, r = 0.5, 0.5, 0.3
    rng = np.random.default_rng(5)
    jet = _poly(rng, 5)
    xi, yi = grid.node_xy(cx, cy, r)
    n = grid.n
    coef = {
        "axx": 2.0 + 0.5 * rng.uniform(size=n), "axy": 0.3 * rng.uniform(-1, 1, n),
        "ayy": 1.5 + 0.5 * rng.uniform(size=n), "bx": rng.standard_normal(n),
        "by": rng.standard_normal(n), "c": -rng.uniform(size=n),
    }
    u, ux, uy, uxx, uxy, uyy = jet(xi, yi)
    Lu = (0.5 * coef["axx"] * uxx + coef["axy"] * uxy + 0.5 * coef["ayy"] * uyy
          + coef["bx"] * ux + coef["by"] * uy + coef["c"] * u)
    A_II, A_IB = grid.collocation(r, coef)
    xb, yb = _ring_xy(grid, cx, cy, r)
    w_B = jet(xb, yb)[0]
    w_I = spectral.solve_refined(A_II, (-A_IB @ w_B - (-Lu))[:, None])[:, 0]
    assert np.max(np.abs(w_I - u)) < 1e-10 * (1 + np.max(np.abs(u)))


def test_disk_harmonic_extension_closed_form():
    # Laplace on the unit disk: ring data cos(k theta) extends to rho^k cos(k theta).
    grid = spectral.local_grid(8, 24)
    n = grid.n
    coef = {"axx": np.full(n, 2.0), "axy": np.zeros(n), "ayy": np.full(n, 2.0),
            "bx": np.zeros(n), "by": np.zeros(n), "c": np.zeros(n)}
    A_II, A_IB = grid.collocation(1.0, coef)
    for k in (0, 1, 5, 11, 12):
        w_B = np.cos(k * grid.theta)
        w_I = np.linalg.solve(A_II, -A_IB @ w_B)
        ref = grid.rho ** k * np.cos(k * grid.th_node)
        assert np.max(np.abs(w_I - ref)) < 1e-11, k


def test_poisson_constant_source_closed_form():
    # Laplacian operator with f constant and zero ring data: B = f (r^2 - d^2) / 4.
    grid = spectral.local_grid(5, 12)
    n = grid.n
    r, f0 = 0.4, 3.0
    coef = {"axx": np.full(n, 2.0), "axy": np.zeros(n), "ayy": np.full(n, 2.0),
            "bx": np.zeros(n), "by": np.zeros(n), "c": np.zeros(n)}
    A_II, _ = grid.collocation(r, coef)
    w = np.linalg.solve(A_II, -np.full(n, f0))
    assert np.max(np.abs(w - f0 * (r * r - (r * grid.rho) ** 2) / 4)) < 1e-13


def _eq46_laplacian():
    sympy = pytest.importorskip("sympy")
    x, y = sympy.symbols("x y", real=True)
    u = (3 + sympy.Rational(1, 3) * sympy.sin(sympy.sqrt(1 + x ** 2 / 100 + y ** 2 / 50))
         + sympy.Rational(1, 3) * sympy.tanh(sympy.sin(3 * x / 25 + y / 20)
                                             + sympy.sin(x / 20 - 3 * y / 25)))
    lap = sympy.diff(u, x, 2) + sympy.diff(u, y, 2)
    return sympy.lambdify((x, y), u, "numpy"), sympy.lambdify((x, y), lap, "numpy")


@pytest.mark.parametrize("centre", [(0.0, 0.0), (40.0, 40.0), (-45.0, 10.0)])
def test_paper_local_solve_example(centre):
    # Section 4: one subdomain of radius about 9 with 44 x 22 nodes solves the
    # local problem of eq. 46 with a maximum error of order 1e-12 and a
    # collocation matrix whose condition number is of order 1e5.
    u_f, lap_f = _eq46_laplacian()
    grid = spectral.local_grid(22, 44)
    n = grid.n
    cx, cy = centre
    r = 9.0
    coef = {"axx": np.full(n, 2.0), "axy": np.zeros(n), "ayy": np.full(n, 2.0),
            "bx": np.zeros(n), "by": np.zeros(n), "c": np.zeros(n)}
    A_II, A_IB = grid.collocation(r, coef)
    xi, yi = grid.node_xy(cx, cy, r)
    xb, yb = _ring_xy(grid, cx, cy, r)
    f_src = -lap_f(xi, yi)      # nabla^2 u = F  <=>  L u + f = 0 with f = -F
    w = spectral.solve_refined(A_II, (-A_IB @ u_f(xb, yb) - f_src)[:, None])[:, 0]
    err = np.max(np.abs(w - u_f(xi, yi)))
    assert err < 5e-11
    # order 1e5 (the reading Nr = 22 interior radii gives 7.7e4 for every centre)
    cond = np.linalg.cond(A_II)
    assert 3e4 < cond < 3e5


def _config1_cover():
    cfg = workloads.config1()
    return cfg, geometry.build_cover(cfg["problem"]["domain"], cfg["cover"])


def test_floating_rows_laplace_closed_form():
    # With Ntheta = M the Laplace rows are the discrete Poisson-kernel series
    # C_ij = -(1/M)[1 + 2 sum_{k<M/2} rho^k cos k(phi - theta_j) + rho^{M/2} cos (M/2)(phi - theta_j)].
    cfg, cv = _config1_cover()
    for m in np.nonzero(cv.floating)[0]:
        knots, Crows, rv = spectral.floating_rows(cfg["problem"], cv, m)
        M = int(cv.M[m])
        thj = 2 * math.pi * np.arange(M) / M
        for t, i in enumerate(knots):
            rho, phi = spectral.knot_polar(cv, m, i)
            x = phi - thj
            ref = 1 + rho ** (M // 2) * np.cos(M / 2 * x)
            for k in range(1, M // 2):
                ref = ref + 2 * rho ** k * np.cos(k * x)
            assert np.max(np.abs(Crows[t] + ref / M)) < 1e-12
            assert abs(rv[t]) < 1e-15


def test_floating_rows_reproduce_harmonic_polynomial_and_sum_to_zero():
    cfg, cv = _config1_cover()
    g = cfg["problem"]["g"]
    for m in np.nonzero(cv.floating)[0]:
        knots, Crows, rv = spectral.floating_rows(cfg["problem"], cv, m)
        st = cv.stencil(m)
        u_st = fields.value(g, cv.knot_xy[st, 0], cv.knot_xy[st, 1])
        u_k = fields.value(g, cv.knot_xy[knots, 0], cv.knot_xy[knots, 1])
        assert np.max(np.abs(u_k + Crows @ u_st - rv)) < 1e-11
        # c = 0: G 1 = 0 on these rows (sum_j H_j = 1 and the solution -1 of eq. 32)
        assert np.max(np.abs(1.0 + Crows.sum(axis=1))) < 1e-11
