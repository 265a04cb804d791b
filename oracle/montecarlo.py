"""Feynman-Kac Monte Carlo estimates of the perimeter rows of C and r
(Section 2.3 eqs. 25-30, Section 2.4 eqs. 36-37, Appendix eq. 53).

For a knot x_i assigned to a perimeter subdomain Omega_m = circle_m cap Omega,
paths of dX = b dt + sigma dW, dY = c Y dt, dZ = f Y dt start at (x_i, 1, 0)
and stop at the first exit from Omega_m.  Then
  C_ij = -E[1_{exit on Gamma_m} H_j(X_tau) Y_tau],  j in Xi_m  (eq. 29)
  r_i  =  E[1_{exit on boundary} g(X_tau) Y_tau + Z_tau]      (eq. 30)
with H_j the inverse-multiquadric cardinal functions of the arc (eq. 22).
Since H_j = sum_l (K^-1)_lj phi_l, the estimator accumulates
S_l = sum_paths 1_Gamma Y phi_l(theta(X_tau)) and applies K^-1 once.

Readings where the paper defers to its reference on the integrator:

* Plain Euler-Maruyama with step h and left-point coefficients.  Step k of
  path p from knot i uses two normals from Philox4x32-10 with counter
  (k, p, i, 0) (see ``philox``).
* A step whose end point stays in Omega_m (strictly inside the circle and in
  Omega) is accepted: Y <- Y exp(c h), Z <- Z + f Y h.  Otherwise the path
  exits at the first crossing t* in (0, 1] of the segment with the circle or
  with a boundary piece that the end point violates; the exit is on Gamma_m
  if the circle is crossed first.  Y and Z advance by the fraction t* of the
  step.
* The exit angle is unwrapped into the arc and clamped to its ends.
* Paths are split into B contiguous batches (batch of path p = p B div Ntilde);
  the standard error of each entry is the standard deviation of the batch
  estimates over sqrt(B).
* More than step_cap steps on one path is an error (the representation
  needs E[tau] < infinity, Appendix).
* Scheme 1 (``mc["scheme"] == 1``): the boundary-shifted Euler scheme of
  Gobet and Menozzi (the paper's ref. [15]; SPA 120 (2010)).  An accepted end
  point q that lies closer to a piece of the boundary of Omega_m (the circle,
  a side of the box, the outer circle or a hole of the disk) than
  c0 sqrt(h) |sigma^T n|, with n the piece's outward normal at q, sigma taken
  at the step's left point and c0 = -zeta(1/2) / sqrt(2 pi), stops the path
  there after the full step; the exit point is q projected onto the nearest
  such piece (ties: the circle first, then the pieces in the order above).
  End points outside Omega_m exit as in scheme 0.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from . import cardinal, fields, philox
from .geometry import ROW_MC, inside

TWO_PI = 2.0 * math.pi
# -zeta(1/2) / sqrt(2 pi): the mean overshoot constant of the shifted scheme
GM_C0 = 0.5825971579390106


class PathCapError(RuntimeError):
    pass


def _exit_circle(px, py, dx, dy, cx, cy, r):
    """Positive root t of |p + t d - c| = r for p strictly inside the circle."""
    a = dx * dx + dy * dy
    ex, ey = px - cx, py - cy
    b = ex * dx + ey * dy
    cc = ex * ex + ey * ey - r * r
    sq = np.sqrt(np.maximum(b * b - a * cc, 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(b > 0.0, -cc / (b + sq), (sq - b) / a)
    return t


def _enter_circle(px, py, dx, dy, cx, cy, r):
    """Smaller positive root of |p + t d - c| = r for p outside the circle."""
    a = dx * dx + dy * dy
    ex, ey = px - cx, py - cy
    b = ex * dx + ey * dy
    cc = ex * ex + ey * ey - r * r
    sq = np.sqrt(np.maximum(b * b - a * cc, 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(b < 0.0, cc / (sq - b), (-b - sq) / a)
    return t


def _exit_domain(dom, px, py, qx, qy):
    """First crossing fraction of segment p -> q with each boundary piece that
    the end point q violates (inf where none)."""
    dx, dy = qx - px, qy - py
    t = np.full(px.shape, np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        if dom["kind"] == "box":
            for bound, coord, d, lower in ((dom["x0"], px, dx, True), (dom["x1"], px, dx, False),
                                           (dom["y0"], py, dy, True), (dom["y1"], py, dy, False)):
                q = coord + d
                viol = (q <= bound) if lower else (q >= bound)
                t = np.where(viol, np.minimum(t, (bound - coord) / d), t)
        else:
            R = dom["R"]
            viol = (qx - dom["cx"]) ** 2 + (qy - dom["cy"]) ** 2 >= R * R
            t = np.where(viol, np.minimum(t, _exit_circle(px, py, dx, dy, dom["cx"], dom["cy"], R)), t)
            for hx, hy, hr in dom["holes"]:
                viol = (qx - hx) ** 2 + (qy - hy) ** 2 <= hr * hr
                t = np.where(viol, np.minimum(t, _enter_circle(px, py, dx, dy, hx, hy, hr)), t)
    return t


def _shift_stops(dom, qx, qy, cx, cy, r, s11, s21, s22, sqh):
    """Scheme 1: for end points q inside Omega_m, whether the path stops
    (q within c0 sqrt(h) |sigma^T n| of a boundary piece), the projection of q
    onto the nearest such piece, and whether that piece is the circle."""
    def band(nx, ny):
        return GM_C0 * sqh * np.sqrt((s11 * nx + s21 * ny) ** 2 + (s22 * ny) ** 2)

    pieces = []      # (distance, normal x, normal y, projection x, projection y, is circle)
    ex, ey = qx - cx, qy - cy
    rho = np.sqrt(ex * ex + ey * ey)
    with np.errstate(divide="ignore", invalid="ignore"):
        nx, ny = ex / rho, ey / rho
    pieces.append((r - rho, nx, ny, cx + r * nx, cy + r * ny, True))
    one, zero = np.ones_like(qx), np.zeros_like(qx)
    if dom["kind"] == "box":
        pieces.append((qx - dom["x0"], -one, zero, np.full_like(qx, dom["x0"]), qy, False))
        pieces.append((dom["x1"] - qx, one, zero, np.full_like(qx, dom["x1"]), qy, False))
        pieces.append((qy - dom["y0"], zero, -one, qx, np.full_like(qy, dom["y0"]), False))
        pieces.append((dom["y1"] - qy, zero, one, qx, np.full_like(qy, dom["y1"]), False))
    else:
        fx, fy = qx - dom["cx"], qy - dom["cy"]
        d = np.sqrt(fx * fx + fy * fy)
        with np.errstate(divide="ignore", invalid="ignore"):
            ux, uy = fx / d, fy / d
        pieces.append((dom["R"] - d, ux, uy, dom["cx"] + dom["R"] * ux, dom["cy"] + dom["R"] * uy, False))
        for hx, hy, hr in dom["holes"]:
            fx, fy = qx - hx, qy - hy
            d = np.sqrt(fx * fx + fy * fy)
            with np.errstate(divide="ignore", invalid="ignore"):
                ux, uy = fx / d, fy / d
            pieces.append((d - hr, -ux, -uy, hx + hr * ux, hy + hr * uy, False))
    best = np.full(qx.shape, np.inf)
    sx, sy = qx.copy(), qy.copy()
    gam = np.zeros(qx.shape, dtype=bool)
    for dist, nx_, ny_, px_, py_, circ in pieces:
        hit = (dist < band(nx_, ny_)) & (dist < best)
        best = np.where(hit, dist, best)
        sx = np.where(hit, px_, sx)
        sy = np.where(hit, py_, sy)
        gam = np.where(hit, circ, gam)
    return np.isfinite(best), sx, sy, gam


def arc_angles(cover, m):
    """Local angles of the stencil knots of perimeter circle m (eq. 12)."""
    return cover.knot_theta[cover.knot_off[m]:cover.knot_off[m + 1]]


def unwrap_to_arc(theta, t0, t1):
    loc = t0 + np.mod(theta - t0, TWO_PI)
    over = loc > t1
    to_hi = (loc - t1) <= (t0 + TWO_PI - loc)
    return np.where(over, np.where(to_hi, t1, t0), loc)


def run_paths(problem, cover, mc, knots):
    """Euler-Maruyama paths of eq. 53 from each of the given knots inside the
    subdomain of its assigned circle, stopped at the first exit.  Returns the
    exit states per path, path-major within knot-major order:
    (x, y, Y, Z, on_Gamma, steps)."""
    dom = problem["domain"]
    P = int(mc["paths"])
    cap = int(mc["step_cap"])
    seed = int(mc["seed"])
    scheme = int(mc.get("scheme", 0))
    knots = np.asarray(knots, dtype=np.int64)
    K = len(knots)
    kk = np.repeat(knots, P)
    pp = np.tile(np.arange(P, dtype=np.int64), K)
    slot = np.repeat(np.arange(K), P)
    mm = cover.assigned[kk]
    cx, cy, rr = cover.centres[mm, 0], cover.centres[mm, 1], cover.radii[mm]
    if mc.get("h_per_circle") is not None:
        hh = np.asarray(mc["h_per_circle"])[mm]
    else:
        hh = np.full(len(kk), float(mc["h"]))
    X = cover.knot_xy[kk, 0].copy()
    Yp = cover.knot_xy[kk, 1].copy()
    Yw = np.ones(len(kk))
    Zw = np.zeros(len(kk))
    ex_x = np.zeros(len(kk))
    ex_y = np.zeros(len(kk))
    ex_Y = np.zeros(len(kk))
    ex_Z = np.zeros(len(kk))
    ex_gamma = np.zeros(len(kk), dtype=bool)
    nsteps = np.zeros(len(kk), dtype=np.int64)
    active = np.arange(len(kk))
    k = 0
    while active.size:
        if k >= cap:
            raise PathCapError(f"{active.size} paths exceeded {cap} steps")
        x, y = X[active], Yp[active]
        h = hh[active]
        n1, n2 = philox.normals(k, pp[active], kk[active], seed)
        co = fields.coefficients(problem, x, y)
        s11, s21, s22 = fields.sigma(co["axx"], co["axy"], co["ayy"])
        sq = np.sqrt(h)
        qx = x + co["bx"] * h + sq * (s11 * n1)
        qy = y + co["by"] * h + sq * (s21 * n1 + s22 * n2)
        ccx, ccy, r = cx[active], cy[active], rr[active]
        in_c = (qx - ccx) ** 2 + (qy - ccy) ** 2 < r * r
        in_d = inside(dom, qx, qy)
        stay = in_c & in_d
        Y0, Z0 = Yw[active], Zw[active]
        if scheme == 1 and stay.any():
            stop, sx, sy, sgam = _shift_stops(dom, qx, qy, ccx, ccy, r, s11, s21, s22, sq)
            stop &= stay
            if stop.any():
                ids = active[stop]
                ex_x[ids] = sx[stop]
                ex_y[ids] = sy[stop]
                ex_Y[ids] = Y0[stop] * np.exp(co["c"][stop] * h[stop])
                ex_Z[ids] = Z0[stop] + co["f"][stop] * Y0[stop] * h[stop]
                ex_gamma[ids] = sgam[stop]
                nsteps[ids] = k + 1
                stay = stay & ~stop
        # accepted steps
        st = active[stay]
        X[st] = qx[stay]
        Yp[st] = qy[stay]
        Yw[st] = Y0[stay] * np.exp(co["c"][stay] * h[stay])
        Zw[st] = Z0[stay] + co["f"][stay] * Y0[stay] * h[stay]
        # exits through the boundary
        e = ~(in_c & in_d)
        if e.any():
            px, py, tqx, tqy = x[e], y[e], qx[e], qy[e]
            dxe, dye = tqx - px, tqy - py
            tc = np.where(in_c[e], np.inf,
                          _exit_circle(px, py, dxe, dye, ccx[e], ccy[e], r[e]))
            td = np.where(in_d[e], np.inf, _exit_domain(dom, px, py, tqx, tqy))
            ts = np.clip(np.minimum(tc, td), 0.0, 1.0)
            ids = active[e]
            he = h[e]
            ex_x[ids] = px + ts * dxe
            ex_y[ids] = py + ts * dye
            ex_Y[ids] = Y0[e] * np.exp(co["c"][e] * ts * he)
            ex_Z[ids] = Z0[e] + co["f"][e] * Y0[e] * ts * he
            ex_gamma[ids] = tc <= td
            nsteps[ids] = k + 1
        active = st
        k += 1
    return ex_x, ex_y, ex_Y, ex_Z, ex_gamma, nsteps


def simulate_knots(problem, cover, mc, knots):
    """Run all paths from the given MC knots.  Returns per-knot, per-batch sums
    S_phi (list of (B, n_arc)), S_g (K, B), batch counts (B,) and path-steps."""
    P = int(mc["paths"])
    B = int(mc["n_batches"])
    knots = np.asarray(knots, dtype=np.int64)
    K = len(knots)
    pp = np.tile(np.arange(P, dtype=np.int64), K)
    slot = np.repeat(np.arange(K), P)
    ex_x, ex_y, ex_Y, ex_Z, ex_gamma, nsteps = run_paths(problem, cover, mc, knots)
    batch = (pp * B) // P
    counts = np.bincount(batch[:P], minlength=B).astype(np.float64)
    gvals = fields.value(problem["g"], ex_x, ex_y, problem)
    pay_g = np.where(ex_gamma, 0.0, gvals * ex_Y) + ex_Z
    S_g = np.zeros((K, B))
    np.add.at(S_g, (slot, batch), pay_g)
    S_phi = []
    for t in range(K):
        i = knots[t]
        m = cover.assigned[i]
        sel = slice(t * P, (t + 1) * P)
        th_l = arc_angles(cover, m)
        t0, t1 = cover.arc[m]
        theta = np.arctan2(ex_y[sel] - cover.centres[m, 1], ex_x[sel] - cover.centres[m, 0])
        theta = unwrap_to_arc(theta, t0, t1)
        w = np.where(ex_gamma[sel], ex_Y[sel], 0.0)
        phi = cardinal.imq(theta[:, None], th_l[None, :], cover.rbf_c2[m])
        Sb = np.zeros((B, len(th_l)))
        np.add.at(Sb, batch[sel], w[:, None] * phi)
        S_phi.append(Sb)
    return S_phi, S_g, counts, int(nsteps.sum())


def finalize(cover, knots, S_phi, S_g, counts):
    """C[i, Xi_m] = -K_m^-1 (S_phi / Ntilde), r_i = S_g / Ntilde, with batch
    standard errors.  Returns lists of (Crow, se_row) and arrays r, se_r."""
    B = len(counts)
    P = counts.sum()
    rows, ses = [], []
    r = np.zeros(len(knots))
    se_r = np.zeros(len(knots))
    for t, i in enumerate(knots):
        m = cover.assigned[i]
        Kg = cardinal.imq_gram(arc_angles(cover, m), cover.rbf_c2[m])
        cho = sla.cho_factor(Kg, lower=True)
        total = -sla.cho_solve(cho, S_phi[t].sum(axis=0) / P)
        per_b = -sla.cho_solve(cho, (S_phi[t] / counts[:, None]).T).T
        rows.append(total)
        ses.append(per_b.std(axis=0, ddof=1) / math.sqrt(B))
        r[t] = S_g[t].sum() / P
        se_r[t] = (S_g[t] / counts).std(ddof=1) / math.sqrt(B)
    return rows, ses, r, se_r


def mc_rows(problem, cover, mc, knots=None, chunk_paths=2_000_000):
    """Perimeter rows for the given knots (default: all MC knots)."""
    if knots is None:
        knots = np.nonzero(cover.row_class == ROW_MC)[0]
    knots = np.asarray(knots, dtype=np.int64)
    P = int(mc["paths"])
    per = max(1, chunk_paths // P)
    rows, ses, rs, sers, steps = [], [], [], [], 0
    for s in range(0, len(knots), per):
        ks = knots[s:s + per]
        S_phi, S_g, counts, st = simulate_knots(problem, cover, mc, ks)
        a, b, c, d = finalize(cover, ks, S_phi, S_g, counts)
        rows += a
        ses += b
        rs.append(c)
        sers.append(d)
        steps += st
    r = np.concatenate(rs) if rs else np.zeros(0)
    se_r = np.concatenate(sers) if sers else np.zeros(0)
    return knots, rows, ses, r, se_r, steps
