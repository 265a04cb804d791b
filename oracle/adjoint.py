"""Exact derivative of the discrete assembly-and-solve map with respect to the
node samples of the coefficients on floating circles (not in the paper).

With R(u, theta) = C u - r = 0 and a loss L(u), dL/dtheta = -lambda^T dR/dtheta
where C^T lambda = dL/du.  For a knot x_i assigned to floating circle m,
(C u - r)_i = u_i - (e_i^T w_I + eps_i^T w_B), where w_B = H u_Xi are the ring
values and w_I = -A_II^-1 (A_IB w_B + F) the interior values of the discrete
local solution (eqs. 32, 35, 40).  Differentiating the collocation equations
A_II w_I + A_IB w_B + F = 0 gives, with mu = A_II^-T E_m^T lambda_{K_m},

  dL/d(coef_q) = -mu_q (Op_coef[q, :] . [w_I; w_B])   for a_xx, a_xy, a_yy, b_x, b_y, c
  dL/d(f_q)    = -mu_q

where Op_coef[q, :] is the operator row that multiplies the coefficient's
sample at node q.  Monte Carlo and boundary rows do not depend on node
samples; their right-hand sides have dL/dr_i = lambda_i.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import assemble, geometry, spectral

COEFS = ("axx", "axy", "ayy", "bx", "by", "c")


def circle_weights(cover, m, grid):
    knots = np.nonzero(cover.assigned == m)[0]
    E = np.zeros((len(knots), grid.n))
    Eps = np.zeros((len(knots), grid.Nt))
    for t, i in enumerate(knots):
        rho, phi = spectral.knot_polar(cover, m, i)
        E[t], Eps[t] = grid.eval_weights(rho, phi)
    return knots, E, Eps


def circle_terms(cover, m, samples, u, lam):
    """The adjoint quantities of floating circle m: mu = A_II^-T E^T lambda_Km,
    the local solution [w_I; w_B] at u, and the coefficient operator rows."""
    grid = spectral.local_grid(cover.Nr[m], cover.Ntheta[m])
    r = float(cover.radii[m])
    A_II, A_IB = grid.collocation(r, samples)
    Mm = int(cover.M[m])
    from . import cardinal
    H = cardinal.fourier_matrix(grid.theta, Mm)
    knots, E, _ = circle_weights(cover, m, grid)
    lu = sla.lu_factor(A_II)
    mu = sla.lu_solve(lu, E.T @ lam[knots], trans=1)
    w_B = H @ u[cover.knot_off[m]:cover.knot_off[m + 1]]
    w_I = -sla.lu_solve(lu, A_IB @ w_B + samples["f"])
    w_full = np.concatenate([w_I, w_B])
    return mu, w_full, grid.coefficient_ops(r)


def circle_gradient(cover, m, samples, u, lam):
    """Gradients of the loss w.r.t. the seven node samples of floating circle m."""
    mu, w_full, ops = circle_terms(cover, m, samples, u, lam)
    g = {name: -mu * (ops[name] @ w_full) for name in COEFS}
    g["f"] = -mu
    return g


def loss_sq(u, target):
    return float(np.sum((u - target) ** 2))


def gradient(problem, cover, system, samples, target):
    """Loss sum (u - target)^2, its gradient w.r.t. every floating circle's
    node samples, and lambda = C^-T dL/du (= dL/dr).  Under rule AVERAGED
    (eqs. 38-39) row i is the sum of its pair rows, so each pair (knot i,
    circle m) enters circle m's terms with the multiplier lambda_i."""
    u = assemble.solve(system)
    lam = assemble.solve(system, rhs=2.0 * (u - target), transpose=True)
    rows, lam_rows = cover, lam
    if cover.containers is not None:
        rows, pknot = geometry.pair_cover(cover)
        lam_rows = lam[pknot]
    grads = {m: circle_gradient(rows, m, samples[m], u, lam_rows)
             for m in np.nonzero(cover.floating)[0]}
    return loss_sq(u, target), grads, lam, u


def loss_after_perturbation(problem, cover, system, samples, target, m, name, q, eps):
    """Loss with sample q of coefficient ``name`` on circle m shifted by eps:
    only the rows assigned to circle m change."""
    s = {k: v.copy() for k, v in samples[m].items()}
    s[name][q] += eps
    knots, Crows, rv = spectral.floating_rows(problem, cover, m, s)
    val = system.val.copy()
    b = system.b.copy()
    for t, i in enumerate(knots):
        assemble._put_row(cover, val, system.se.copy(), i, m, Crows[t])
        b[i] = rv[t]
    pert = assemble.System(cover, val, b, system.se, system.se_b, 0)
    return loss_sq(assemble.solve(pert), target)
