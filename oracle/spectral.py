"""Polar Chebyshev x Fourier collocation of the local problems on floating
circles and the floating rows of C and r (Section 2.4 eqs. 31-35, Section 3.3
eqs. 40-41).

Readings where the paper only cites a textbook recipe:

* Radial grid: Chebyshev-Gauss-Lobatto points x_j = cos(j pi / Nc),
  j = 0..Nc, with Nc = 2 Nr + 1 odd, on the full diameter [-1, 1]; x_0 = 1 is
  the ring, x_1..x_Nr are the Nr interior radii (no node at the centre).
  Values at negative x are read through u(-rho, theta) = u(rho, theta + pi).
* Angular grid: theta_l = 2 pi l / Ntheta, Ntheta even.
* Unknowns: n = Nr Ntheta interior values ordered q = (j - 1) Ntheta + l.
* Derivatives: the Chebyshev differentiation matrix (and its square) along
  the diameter, the derivatives of the eq.-18 cardinal functions along the
  angle, combined through the polar chain rule on a circle of radius r.
* The collocation matrix is split as [A_II | A_IB] (interior | ring); the
  ring values are eliminated into the right-hand sides.  Row i of C for a
  knot x_i assigned to circle m: C[i, Xi_m] = e_i^T W[:, :M] - eps_i^T H and
  r_i = e_i^T W[:, M], with W = A_II^-1 [A_IB H | -F], H the M-knot cardinal
  functions at the ring angles, and (e_i, eps_i) the interpolation weights of
  x_i over interior and ring values.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from . import cardinal, fields


# ---------------------------------------------------------------------------
# One-dimensional operators
# ---------------------------------------------------------------------------

def cheb_points(Nc):
    return np.cos(np.pi * np.arange(Nc + 1) / Nc)


def lagrange_weights(x):
    """Barycentric weights w_j = 1 / prod_{k != j} (x_j - x_k), from the definition."""
    n = len(x)
    w = np.ones(n)
    for j in range(n):
        for k in range(n):
            if k != j:
                w[j] /= (x[j] - x[k])
    return w


def lagrange_diff(x):
    """D[i, j] = l_j'(x_i) for the Lagrange basis on nodes x:
    l_j'(x_i) = (w_j / w_i) / (x_i - x_j) for i != j, l_i'(x_i) = sum_{k != i} 1 / (x_i - x_k)."""
    n = len(x)
    w = lagrange_weights(x)
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (w[j] / w[i]) / (x[i] - x[j])
        D[i, i] = sum(1.0 / (x[i] - x[k]) for k in range(n) if k != i)
    return D


def lagrange_eval(x, t):
    """l_j(t) for all j, from the product definition."""
    n = len(x)
    out = np.ones(n)
    for j in range(n):
        for k in range(n):
            if k != j:
                out[j] *= (t - x[k]) / (x[j] - x[k])
    return out


def fourier_diff(Nt):
    """D1[l, l'] = d/dtheta of the eq.-18 cardinal H_l' at theta_l; D2 the second derivative."""
    th = 2.0 * np.pi * np.arange(Nt) / Nt
    d1, d2 = cardinal.fourier_cardinal_derivs(th[:, None], th[None, :], Nt)
    return d1, d2


# ---------------------------------------------------------------------------
# Collocation on one floating circle
# ---------------------------------------------------------------------------

class LocalGrid:
    """Grid, fold and unit polar operators for given (Nr, Ntheta)."""

    def __init__(self, Nr, Nt):
        self.Nr, self.Nt = int(Nr), int(Nt)
        self.Nc = 2 * self.Nr + 1
        self.x = cheb_points(self.Nc)
        self.theta = 2.0 * np.pi * np.arange(self.Nt) / self.Nt
        self.n = self.Nr * self.Nt
        Dx = lagrange_diff(self.x)
        Dt1, Dt2 = fourier_diff(self.Nt)
        Ix = np.eye(self.Nc + 1)
        It = np.eye(self.Nt)
        # Operators on the full (Nc + 1) x Nt grid (index J = j Nt + l), kept
        # only at the interior rows j = 1..Nr, then folded onto the unknowns.
        inner = slice(1, self.Nr + 1)
        self.fold = self._fold()
        full_rows = {
            "rr": np.kron((Dx @ Dx)[inner], It),
            "r": np.kron(Dx[inner], It),
            "tt": np.kron(Ix[inner], Dt2),
            "t": np.kron(Ix[inner], Dt1),
            "rt": np.kron(Dx[inner], Dt1),
        }
        self.unit = {k: v @ self.fold for k, v in full_rows.items()}
        # node polar coordinates (interior only)
        self.rho = np.repeat(self.x[1:self.Nr + 1], self.Nt)
        self.th_node = np.tile(self.theta, self.Nr)

    def _fold(self):
        """Full-grid values from [interior unknowns (n) | ring values (Nt)]."""
        Nr, Nt, Nc = self.Nr, self.Nt, self.Nc
        P = np.zeros(((Nc + 1) * Nt, self.n + Nt))
        half = Nt // 2
        for j in range(Nc + 1):
            for l in range(Nt):
                J = j * Nt + l
                if j == 0:
                    P[J, self.n + l] = 1.0
                elif j <= Nr:
                    P[J, (j - 1) * Nt + l] = 1.0
                elif j < Nc:
                    k = Nc - j
                    P[J, (k - 1) * Nt + (l + half) % Nt] = 1.0
                else:
                    P[J, self.n + (l + half) % Nt] = 1.0
        return P

    def node_xy(self, cx, cy, r):
        return (cx + r * self.rho * np.cos(self.th_node),
                cy + r * self.rho * np.sin(self.th_node))

    def physical_ops(self, r):
        """Polar chain rule on a circle of radius r: operators (n x (n + Nt)) for
        d_xx, d_xy, d_yy, d_x, d_y acting on [interior | ring] values."""
        C = np.cos(self.th_node)[:, None]
        S = np.sin(self.th_node)[:, None]
        rho = self.rho[:, None]
        U = self.unit
        dxx = (C * C * U["rr"] + S * S / rho * U["r"] + S * S / rho ** 2 * U["tt"]
               - 2 * S * C / rho * U["rt"] + 2 * S * C / rho ** 2 * U["t"]) / r ** 2
        dyy = (S * S * U["rr"] + C * C / rho * U["r"] + C * C / rho ** 2 * U["tt"]
               + 2 * S * C / rho * U["rt"] - 2 * S * C / rho ** 2 * U["t"]) / r ** 2
        dxy = (S * C * U["rr"] - S * C / rho * U["r"] - S * C / rho ** 2 * U["tt"]
               + (C * C - S * S) / rho * U["rt"] - (C * C - S * S) / rho ** 2 * U["t"]) / r ** 2
        dx = (C * U["r"] - S / rho * U["t"]) / r
        dy = (S * U["r"] + C / rho * U["t"]) / r
        return {"xx": dxx, "xy": dxy, "yy": dyy, "x": dx, "y": dy}

    def coefficient_ops(self, r):
        """d(row q of [A_II | A_IB]) / d(sample q of each coefficient): the
        operator rows that multiply a_xx, a_xy, a_yy, b_x, b_y and c in eq. 1."""
        P = self.physical_ops(r)
        ident = np.hstack([np.eye(self.n), np.zeros((self.n, self.Nt))])
        return {"axx": 0.5 * P["xx"], "axy": P["xy"], "ayy": 0.5 * P["yy"],
                "bx": P["x"], "by": P["y"], "c": ident}

    def collocation(self, r, coef):
        """[A_II | A_IB] = sum over coefficients of diag(samples) * operator rows."""
        ops = self.coefficient_ops(r)
        A = np.zeros((self.n, self.n + self.Nt))
        for name, op in ops.items():
            A += coef[name][:, None] * op
        return A[:, :self.n], A[:, self.n:]

    def eval_weights(self, rho, phi):
        """Interpolation weights (e over interior unknowns, eps over the ring) of
        the full-grid interpolant at polar point (rho, phi), rho in [0, 1)."""
        lx = lagrange_eval(self.x, rho)
        lt = cardinal.fourier_cardinal(phi, self.theta, self.Nt)
        full = np.outer(lx, lt).ravel()
        w = full @ self.fold
        return w[:self.n], w[self.n:]


_GRIDS = {}


def local_grid(Nr, Nt):
    key = (int(Nr), int(Nt))
    if key not in _GRIDS:
        _GRIDS[key] = LocalGrid(*key)
    return _GRIDS[key]


def solve_refined(A, R):
    """Dense solve of A W = R: LU with partial pivoting (LAPACK getrf) after row
    equilibration, plus one step of float64 iterative refinement."""
    s = 1.0 / np.max(np.abs(A), axis=1)
    As = A * s[:, None]
    lu = sla.lu_factor(As)
    W = sla.lu_solve(lu, R * s[:, None])
    resid = R - A @ W
    W = W + sla.lu_solve(lu, resid * s[:, None])
    return W


def node_samples(problem, grid, cx, cy, r):
    x, y = grid.node_xy(cx, cy, r)
    return fields.coefficients(problem, x, y)


def floating_circle(cover, m, samples):
    """Local solves of eqs. 32 and 35 on floating circle m, given the seven node
    samples.  Returns (W, H, grid, A_II, A_IB) with W = A_II^-1 [A_IB H | -F]."""
    grid = local_grid(cover.Nr[m], cover.Ntheta[m])
    r = float(cover.radii[m])
    A_II, A_IB = grid.collocation(r, samples)
    Mm = int(cover.M[m])
    H = cardinal.fourier_matrix(grid.theta, Mm)          # (Nt, M)
    R = np.hstack([A_IB @ H, -samples["f"][:, None]])
    W = solve_refined(A_II, R)
    return W, H, grid, A_II, A_IB


def knot_polar(cover, m, i):
    cx, cy = cover.centres[m]
    dx, dy = cover.knot_xy[i, 0] - cx, cover.knot_xy[i, 1] - cy
    return math.sqrt(dx * dx + dy * dy) / cover.radii[m], math.atan2(dy, dx)


def floating_rows(problem, cover, m, samples=None):
    """Rows of C (stencil part) and r for the knots assigned to floating circle m
    (eqs. 33 and 35 evaluated at the knots).  Returns (knot ids, Crows (K, M), r (K,))."""
    if samples is None:
        grid = local_grid(cover.Nr[m], cover.Ntheta[m])
        samples = node_samples(problem, grid, *cover.centres[m], cover.radii[m])
    W, H, grid, _, _ = floating_circle(cover, m, samples)
    Mm = int(cover.M[m])
    knots = np.nonzero(cover.assigned == m)[0]
    Crows = np.zeros((len(knots), Mm))
    rvals = np.zeros(len(knots))
    for t, i in enumerate(knots):
        rho, phi = knot_polar(cover, m, i)
        e, eps = grid.eval_weights(rho, phi)
        Crows[t] = e @ W[:, :Mm] - eps @ H
        rvals[t] = e @ W[:, Mm]
    return knots, Crows, rvals
