"""Pins for the oracle's Feynman-Kac Monte Carlo rows (eqs. 25-30, 53)."""
import math

import numpy as np
import pytest

import workloads
from oracle import assemble, cardinal, fields, geometry, montecarlo, philox
from oracle.geometry import ROW_MC


def _disk_setup(r, rho0):
    """One circle deep inside a large box, run through the Monte Carlo path
    routine with a single start point, so that the exit laws of Brownian
    motion in a disk apply."""
    from types import SimpleNamespace
    dom = workloads.box(-50, 50, -50, 50)
    prob = workloads.laplace_problem(dom, workloads.const(0.0))
    cv = SimpleNamespace(centres=np.zeros((1, 2)), radii=np.array([r]),
                         assigned=np.array([0]), knot_xy=np.array([[rho0, 0.0]]))
    return prob, cv


def test_mean_exit_time_in_a_disk():
    # generator = Laplacian (sigma = sqrt 2): E[tau] = (r^2 - rho^2) / 4
    r, rho0, h, P = 0.1, 0.05, 2.5e-6, 4000
    prob, cv = _disk_setup(r, rho0)
    mc = workloads.mc_opts(P, h, seed=9, n_batches=8)
    ex = montecarlo.run_paths(prob, cv, mc, [0])
    tau = ex[5] * h
    exact = (r * r - rho0 * rho0) / 4
    # Euler exit detection overestimates tau by O(sqrt h)
    assert abs(tau.mean() - exact) / exact < 0.12
    assert np.all(ex[4])                                   # every exit on the circle
    assert np.max(np.abs(np.hypot(ex[0], ex[1]) - r)) < 1e-14


def test_exit_angle_follows_poisson_kernel():
    # exit-angle density (r^2 - rho^2) / (2 pi (r^2 - 2 r rho cos t + rho^2))
    r, rho0, h, P = 1.0, 0.6, 4e-5, 6000
    prob, cv = _disk_setup(r, rho0)
    mc = workloads.mc_opts(P, h, seed=4, n_batches=8)
    ex = montecarlo.run_paths(prob, cv, mc, [0])
    t = np.sort(np.mod(np.arctan2(ex[1], ex[0]) + math.pi, 2 * math.pi) - math.pi)
    grid = np.linspace(-math.pi, math.pi, 20001)
    dens = (r * r - rho0 ** 2) / (2 * math.pi * (r * r - 2 * r * rho0 * np.cos(grid) + rho0 ** 2))
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(grid))])
    emp = np.arange(1, P + 1) / P
    ks = np.max(np.abs(np.interp(t, grid, cdf) - emp))
    assert ks < 1.63 / math.sqrt(P) + 0.01                 # 1 % KS level + Euler bias


def test_constant_data_rows_sum_to_rhs():
    # c = f = 0 and g = 1: per path the payoff is 1 on the boundary and
    # sum_j H_j = 1 (to the IMQ partition-of-unity error) on Gamma, so C 1 = r.
    cfg = workloads.config1(paths=200)
    prob = workloads.laplace_problem(workloads.box(), workloads.const(1.0))
    cv = geometry.build_cover(prob["domain"], cfg["cover"])
    knots, rows, ses, rv, se_r, steps = montecarlo.mc_rows(prob, cv, cfg["mc"])
    for t, i in enumerate(knots):
        assert abs(1.0 + rows[t].sum() - rv[t]) < 2e-4


def test_harmonic_polynomial_residual_is_statistical():
    cfg = workloads.config1(paths=1000)
    prob = cfg["problem"]
    cv = geometry.build_cover(prob["domain"], cfg["cover"])
    knots, rows, ses, rv, se_r, steps = montecarlo.mc_rows(prob, cv, cfg["mc"])
    g = prob["g"]
    z = []
    for t, i in enumerate(knots):
        st = cv.stencil(cv.assigned[i])
        u_st = fields.value(g, cv.knot_xy[st, 0], cv.knot_xy[st, 1])
        res = fields.value(g, *cv.knot_xy[i]) + rows[t] @ u_st - rv[t]
        # combined standard error (entries are correlated; sum of |se| bounds it)
        se = se_r[t] + np.sum(np.abs(ses[t] * u_st))
        z.append(abs(res) / se)
    z = np.array(z)
    # the Euler exit bias adds to the statistical error; most rows stay within 3
    assert np.mean(z < 3) > 0.9


def test_weights_are_in_unit_interval_with_nonpositive_c():
    # c <= 0 implies 0 < Y <= 1 (Appendix, eq. 55): with g = 1, f = 0, c = -5
    # the boundary payoff of every path is in (0, 1].
    cfg = workloads.config1(paths=100)
    prob = workloads.laplace_problem(workloads.box(), workloads.const(1.0))
    prob["c"] = workloads.const(-5.0)
    cv = geometry.build_cover(prob["domain"], cfg["cover"])
    knots = np.nonzero(cv.row_class == ROW_MC)[0][:5]
    S_phi, S_g, counts, steps = montecarlo.simulate_knots(prob, cv, cfg["mc"], knots)
    assert np.all(S_g >= 0) and np.all(S_g <= counts[None, :] + 1e-12)
    assert all(np.all(s >= 0) for s in S_phi)


def test_stream_is_deterministic_and_seed_dependent():
    cfg = workloads.config1(paths=64)
    prob = cfg["problem"]
    cv = geometry.build_cover(prob["domain"], cfg["cover"])
    k = np.nonzero(cv.row_class == ROW_MC)[0][:3]
    a = montecarlo.simulate_knots(prob, cv, cfg["mc"], k)
    b = montecarlo.simulate_knots(prob, cv, cfg["mc"], k)
    assert np.array_equal(a[1], b[1]) and a[3] == b[3]
    mc2 = dict(cfg["mc"], seed=cfg["mc"]["seed"] + 1)
    c = montecarlo.simulate_knots(prob, cv, mc2, k)
    assert not np.array_equal(a[1], c[1])


def test_anisotropic_drift_exit_law_of_an_exponential_harmonic():
    # Constant a with a_xy != 0 and constant drift b chosen so that
    # u = exp(k . x) solves L u = 1/2 k^T a k u + (b . k) u = 0 (eq. 1 with
    # c = f = 0): optional stopping gives E[u(X_tau)] = u(x_0) exactly for the
    # diffusion of eq. 53 with sigma the Cholesky factor of a (eq. 3).  The
    # Euler estimate differs by the O(sqrt h) exit bias plus statistics; a
    # wrong sigma (a_xy sign or position) or drift moves it by >10 SE.
    from types import SimpleNamespace
    axx, axy, ayy = 2.0, 0.9, 1.0
    k = np.array([6.0, -4.0])
    b = -0.5 * (axx * k[0] ** 2 + 2 * axy * k[0] * k[1] + ayy * k[1] ** 2) * k / (k @ k)
    prob = workloads.laplace_problem(workloads.box(-50, 50, -50, 50), workloads.const(0.0))
    prob.update(axx=workloads.const(axx), axy=workloads.const(axy), ayy=workloads.const(ayy),
                bx=workloads.const(b[0]), by=workloads.const(b[1]))
    r, x0 = 0.1, np.array([0.03, -0.02])
    cv = SimpleNamespace(centres=np.zeros((1, 2)), radii=np.array([r]), assigned=np.array([0]),
                         knot_xy=x0[None])
    P = 4000
    ex = montecarlo.run_paths(prob, cv, workloads.mc_opts(P, 1e-5, seed=21, n_batches=8), [0])
    uu = np.exp(k[0] * ex[0] + k[1] * ex[1])
    exact = math.exp(k @ x0)
    se = uu.std(ddof=1) / math.sqrt(P)
    assert abs(uu.mean() - exact) <= 3 * se + 2e-3 * exact


@pytest.mark.slow
def test_variable_coefficient_rows_converge_under_step_refinement():
    # small_variable: drift b, a_xy != 0, a variable clipped c and the derived
    # source f (eqs. 1-3 with the SDE of eq. 53 and the estimators of eqs.
    # 29-30).  Applied to the manufactured u, the Monte Carlo rows leave the
    # Euler bias (O(sqrt h)), the IMQ interpolation error and the statistical
    # error.  Over three 4x refinements of h the RMS residual falls each time,
    # by more than 6x in all (2x per level expected), ends below 0.05 and every
    # row is within 3 standard errors.  A drift of the wrong sign in the paths
    # (f unchanged) leaves an RMS of about 0.11 at the finest h.
    cfg = workloads.small_variable()
    prob = cfg["problem"]
    cv = geometry.build_cover(prob["domain"], cfg["cover"])
    mck = np.nonzero(cv.row_class == ROW_MC)[0]
    ks = np.random.default_rng(1).choice(mck, 6, replace=False)
    u = prob["u_exact"]
    rms = []
    for h in (1e-3, 2.5e-4, 6.25e-5, 1.5625e-5):
        mc = workloads.mc_opts(2000, h, seed=7, n_batches=16)
        knots, rows, ses, rv, se_r, steps = montecarlo.mc_rows(prob, cv, mc, ks)
        res, z = [], []
        for t, i in enumerate(knots):
            st = cv.stencil(cv.assigned[i])
            u_st = fields.value(u, cv.knot_xy[st, 0], cv.knot_xy[st, 1])
            r = fields.value(u, *cv.knot_xy[i]) + rows[t] @ u_st - rv[t]
            res.append(r)
            z.append(abs(r) / (se_r[t] + np.sum(np.abs(ses[t] * u_st))))
        rms.append(float(np.sqrt(np.mean(np.square(res)))))
    assert all(b < a for a, b in zip(rms, rms[1:])), rms
    assert rms[-1] < rms[0] / 6 and rms[-1] < 0.05, rms
    assert max(z) < 3, z
