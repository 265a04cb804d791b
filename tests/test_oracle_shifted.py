"""Pins for the oracle's boundary-shifted Euler scheme (Gobet-Menozzi, the
paper's ref. [15]; used for the perimeter rows in Section 4).

* Mean exit time of a disk: with a = 2 I the generator is the Laplacian, so
  E[tau] = (r^2 - |x0 - c|^2) / 4 in closed form.  Plain Euler overestimates
  it by O(sqrt h) (exits between steps are missed); the shifted scheme must
  remove that bias to within the statistical error.
* A harmonic payoff u(X_tau) has mean u(x0); on a circle cut by a box side the
  plain scheme's exit bias shows and the shifted scheme's does not.
* Every stopped path ends on the boundary: on the circle for interface exits,
  on a box side otherwise.
"""
import types

import numpy as np
import pytest

import workloads
from oracle import montecarlo


def _one_circle(cx, cy, r, x0, y0):
    return types.SimpleNamespace(assigned=np.array([0]), centres=np.array([[cx, cy]]),
                                 radii=np.array([r]), knot_xy=np.array([[x0, y0]]))


def _mc(scheme, h=0.01, paths=40000):
    return dict(paths=paths, h=h, seed=3, n_batches=16, step_cap=1 << 20, scheme=scheme)


def test_shifted_scheme_removes_the_exit_time_bias():
    prob = workloads.laplace_problem(workloads.box(-5, 5, -5, 5), workloads.const(0.0))
    prob["f"] = workloads.const(1.0)           # Z_tau = tau
    cv = _one_circle(0.0, 0.0, 1.0, 0.5, 0.0)
    exact = (1.0 - 0.25) / 4.0
    out = {}
    for scheme in (0, 1):
        _, _, _, Z, _, _ = montecarlo.run_paths(prob, cv, _mc(scheme), [0])
        out[scheme] = (Z.mean() - exact, Z.std() / np.sqrt(len(Z)))
    bias0, se0 = out[0]
    bias1, se1 = out[1]
    assert bias0 > 20 * se0                    # O(sqrt h) overshoot of plain Euler
    assert abs(bias1) <= 3 * se1
    assert abs(bias1) < 0.1 * bias0


def test_shifted_scheme_removes_the_harmonic_exit_bias():
    prob = workloads.laplace_problem(workloads.box(-5, 5, -5, 5), workloads.const(0.0))
    cv = _one_circle(4.6, 0.0, 1.0, 4.5, 0.2)  # the circle crosses the side x = 5
    u = lambda x, y: x * x - y * y + 0.5 * x * y
    res = {}
    for scheme in (0, 1):
        x, y, _, _, gam, _ = montecarlo.run_paths(prob, cv, _mc(scheme), [0])
        v = u(x, y)
        res[scheme] = (v.mean() - u(4.5, 0.2), v.std() / np.sqrt(len(v)))
        assert 0.3 < gam.mean() < 0.8
    assert abs(res[0][0]) > 3 * res[0][1]
    assert abs(res[1][0]) <= 2 * res[1][1]


def test_stopped_paths_end_on_the_boundary():
    prob = workloads.laplace_problem(workloads.box(-5, 5, -5, 5), workloads.const(0.0))
    cv = _one_circle(4.6, 0.0, 1.0, 4.5, 0.2)
    x, y, _, _, gam, _ = montecarlo.run_paths(prob, cv, _mc(1, paths=4000), [0])
    rho = np.hypot(x - 4.6, y)
    assert np.all(np.abs(rho[gam] - 1.0) <= 1e-12)
    assert np.all(np.abs(x[~gam] - 5.0) <= 1e-12)
    assert np.all(rho[~gam] <= 1.0 + 1e-12)


def test_default_scheme_is_plain_euler():
    prob = workloads.laplace_problem(workloads.box(-5, 5, -5, 5), workloads.const(0.0))
    cv = _one_circle(4.6, 0.0, 1.0, 4.5, 0.2)
    a = montecarlo.run_paths(prob, cv, {k: v for k, v in _mc(0, paths=500).items() if k != "scheme"}, [0])
    b = montecarlo.run_paths(prob, cv, _mc(0, paths=500), [0])
    for s, t in zip(a, b):
        assert np.array_equal(s, t)
