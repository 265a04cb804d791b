"""Pins for the oracle's assembled system (eqs. 28-30), its solve and its adjoint."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads
from oracle import adjoint, assemble, fields, geometry, spectral
from oracle.geometry import ROW_BOUNDARY, ROW_MC, ROW_SPECTRAL


@pytest.fixture(scope="module")
def c1_system():
    cfg = workloads.config1(paths=400)
    prob = cfg["problem"]
    cv = geometry.build_cover(prob["domain"], cfg["cover"])
    return cfg, cv, assemble.assemble(prob, cv, cfg["mc"])


def test_rows_follow_eq29(c1_system):
    cfg, cv, sysm = c1_system
    A = sysm.matrix().toarray()
    assert np.all(np.diag(A) == 1.0)
    g = cfg["problem"]["g"]
    bnd = cv.row_class == ROW_BOUNDARY
    assert np.allclose(sysm.b[bnd], fields.value(g, cv.knot_xy[bnd, 0], cv.knot_xy[bnd, 1]))
    ue = fields.value(g, cv.knot_xy[:, 0], cv.knot_xy[:, 1])
    res = A @ ue - sysm.b
    assert np.max(np.abs(res[cv.row_class == ROW_SPECTRAL])) < 1e-11
    assert np.all(sysm.se[cv.rowptr[:-1][cv.row_class == ROW_SPECTRAL]] == 0)


def test_sparse_solve_matches_dense(c1_system):
    cfg, cv, sysm = c1_system
    u = assemble.solve(sysm)
    ud = np.linalg.solve(sysm.matrix().toarray(), sysm.b)
    assert np.max(np.abs(u - ud)) < 1e-12 * np.max(np.abs(ud))
    ut = assemble.solve(sysm, rhs=sysm.b, transpose=True)
    assert np.max(np.abs(ut - np.linalg.solve(sysm.matrix().toarray().T, sysm.b))) < 1e-10


def test_diagnostics_resemble_table1_structure(c1_system):
    # Table 1 reports rho(C - I) < 1 and small positive max off-diagonal entries
    cfg, cv, sysm = c1_system
    d = assemble.diagnostics(sysm)
    assert d["rho_C_minus_I"] < 1.0
    assert 0.0 < d["max_offdiag"] < 0.1


@pytest.fixture(scope="module")
def small_var():
    cfg = workloads.small_variable(paths=64)
    prob = cfg["problem"]
    cv = geometry.build_cover(prob["domain"], cfg["cover"])
    samples = {}
    for m in np.nonzero(cv.floating)[0]:
        grid = spectral.local_grid(cv.Nr[m], cv.Ntheta[m])
        samples[m] = spectral.node_samples(prob, grid, *cv.centres[m], cv.radii[m])
    sysm = assemble.assemble(prob, cv, cfg["mc"], samples=samples)
    ue = fields.value(prob["u_exact"], cv.knot_xy[:, 0], cv.knot_xy[:, 1])
    target = ue + np.random.default_rng(0).normal(0, 1e-3, cv.N)
    return prob, cv, sysm, samples, target


def test_adjoint_matches_central_differences(small_var):
    prob, cv, sysm, samples, target = small_var
    L, grads, lam, u = adjoint.gradient(prob, cv, sysm, samples, target)
    rng = np.random.default_rng(11)
    fl = list(samples)
    names = ["axx", "axy", "ayy", "bx", "by", "c", "f"]
    gmax = max(np.max(np.abs(g[k])) for g in grads.values() for k in names)
    for _ in range(12):
        m = fl[rng.integers(len(fl))]
        name = names[rng.integers(len(names))]
        q = int(rng.integers(len(samples[m][name])))
        eps = 1e-5 * max(1.0, abs(samples[m][name][q]))
        Lp = adjoint.loss_after_perturbation(prob, cv, sysm, samples, target, m, name, q, eps)
        Lm = adjoint.loss_after_perturbation(prob, cv, sysm, samples, target, m, name, q, -eps)
        fd = (Lp - Lm) / (2 * eps)
        ga = grads[m][name][q]
        # rounding in the loss (about 1e-13 here) divided by 2 eps sets the floor
        assert abs(fd - ga) <= 1e-5 * abs(ga) + 1e-8 * gmax, (m, name, q, fd, ga)


def test_adjoint_dot_product_identity(small_var):
    # <J v, lambda> = <v, J^T lambda> for a random direction v in the samples of
    # one circle, J = d(C u - r)/d(samples) at fixed u (central differences).
    prob, cv, sysm, samples, target = small_var
    L, grads, lam, u = adjoint.gradient(prob, cv, sysm, samples, target)
    m = list(samples)[0]
    rng = np.random.default_rng(2)
    v = {k: rng.standard_normal(len(s)) for k, s in samples[m].items()}
    eps = 1e-6

    def residual(sign):
        s = {k: samples[m][k] + sign * eps * v[k] for k in v}
        knots, Crows, rv = spectral.floating_rows(prob, cv, m, s)
        st = cv.stencil(m)
        return knots, u[knots] + Crows @ u[st] - rv

    knots, rp = residual(+1)
    _, rm = residual(-1)
    Jv = (rp - rm) / (2 * eps)
    lhs = float(Jv @ lam[knots])
    rhs = -sum(float(grads[m][k] @ v[k]) for k in v)
    assert abs(lhs - rhs) < 1e-6 * (abs(lhs) + abs(rhs))


def test_config2_floating_rows_annihilate_the_manufactured_solution():
    # Variable a, b, clipped c and the derived source (eqs. 1-3) on the 32x32
    # benchmark cover, n = 1024: collocation is spectrally accurate for the
    # smooth manufactured u, so the floating rows (eqs. 31-35) applied to u at
    # the knots leave rounding-level residuals.  This ties derived_source (the
    # operator of eq. 1 applied analytically) to the collocation operator of
    # eq. 40 built from node samples; a dropped term, a wrong factor or sign
    # leaves residuals of order r^2 |f error| >> 1e-10.  First, last and a
    # seeded sample of the 900 floating circles.
    cfg = workloads.config2()
    prob = cfg["problem"]
    cv = geometry.build_cover(prob["domain"], cfg["cover"])
    fl = np.nonzero(cv.floating)[0]
    rng = np.random.default_rng(22)
    sel = np.concatenate([fl[:2], fl[-2:], rng.choice(fl[2:-2], 8, replace=False)])
    u = prob["u_exact"]
    worst = 0.0
    for m in sel:
        knots, Crows, rv = spectral.floating_rows(prob, cv, m)
        st = cv.stencil(m)
        u_st = fields.value(u, cv.knot_xy[st, 0], cv.knot_xy[st, 1])
        for t, i in enumerate(knots):
            worst = max(worst, abs(fields.value(u, *cv.knot_xy[i]) + Crows[t] @ u_st - rv[t]))
    assert worst <= 1e-10, worst
