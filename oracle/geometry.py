"""Cover, subdomains, interfaces, knots, stencils and row choice
(Section 2.1, eqs. 4-12; Section 3.2).

Readings taken where the paper leaves details open:

* A circle is floating when its closed disk lies inside Omega (distance from
  the centre to the boundary exceeds r by more than 1e-12 r); otherwise it is
  a perimeter circle, whose interface is the single arc of the circle inside
  the closure of Omega (eqs. 8, 11).  A circle whose interface is not one arc
  is rejected.
* Floating knots: theta_j = 2 pi j / M, j = 0..M-1 (equispaced, offset 0).
* Perimeter knots: the same global grid restricted to the open arc, minus
  grid angles within dtheta / 4 of an arc end, plus one knot at each junction
  of the arc with the boundary (Section 2.1 requires those).  Junction knots
  lie on the boundary and carry the Dirichlet value (row C_ii = 1, r_i = g).
* Knots are numbered circle by circle in local angular order (eq. 12), so the
  stencil of circle m (eq. 9) is a contiguous index range.
* Row choice (Section 3.2 advises the subdomain whose interface is farthest
  from the knot): among circles containing the knot strictly (depth
  r_m - |x - c_m| > 1e-9 r_m), take the floating one of largest depth; only
  if there is none, the perimeter one of largest depth.  A later candidate
  replaces the current one only if it is deeper by more than 1e-12 r, so
  exact ties go to the lower circle index.  Rule MAX_DEPTH ignores the
  floating/perimeter preference.
* Rule AVERAGED (eqs. 38-39): row i sums the expectations of every circle that
  contains the knot strictly (the same depth test), and C_ii is their number.
  ``containers[i]`` lists them by circle index; ``assigned`` still names the
  circle the default rule would choose.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import cKDTree

ROW_SPECTRAL = 0
ROW_MC = 1
ROW_BOUNDARY = 2

RULE_AVERAGED = 2

TWO_PI = 2.0 * math.pi


class CoverError(ValueError):
    pass


# ---------------------------------------------------------------------------
# Domain
# ---------------------------------------------------------------------------

def signed_distance(dom, x, y):
    """Distance to the boundary, positive inside Omega (exact for inside points)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if dom["kind"] == "box":
        return np.minimum(np.minimum(x - dom["x0"], dom["x1"] - x),
                          np.minimum(y - dom["y0"], dom["y1"] - y))
    if dom["kind"] == "disk":
        d = dom["R"] - np.sqrt((x - dom["cx"]) ** 2 + (y - dom["cy"]) ** 2)
        for hx, hy, hr in dom["holes"]:
            d = np.minimum(d, np.sqrt((x - hx) ** 2 + (y - hy) ** 2) - hr)
        return d
    raise ValueError(dom["kind"])


def inside(dom, x, y):
    return signed_distance(dom, x, y) > 0.0


def boundary_crossings(dom, cx, cy, r):
    """Angles (in [0, 2 pi)) where the circle of centre (cx, cy) and radius r
    meets the boundary of Omega."""
    out = []
    if dom["kind"] == "box":
        for xs in (dom["x0"], dom["x1"]):
            t = (xs - cx) / r
            if abs(t) < 1.0:
                a = math.acos(t)
                out += [a, -a]
        for ys in (dom["y0"], dom["y1"]):
            t = (ys - cy) / r
            if abs(t) < 1.0:
                a = math.asin(t)
                out += [a, math.pi - a]
    else:
        circles = [(dom["cx"], dom["cy"], dom["R"])] + list(dom["holes"])
        for bx, by, br in circles:
            dx, dy = bx - cx, by - cy
            d = math.sqrt(dx * dx + dy * dy)
            if abs(r - br) < d < r + br:
                alpha = math.atan2(dy, dx)
                beta = math.acos((r * r + d * d - br * br) / (2.0 * r * d))
                out += [alpha + beta, alpha - beta]
    return sorted(a % TWO_PI for a in out)


def interface_arc(dom, cx, cy, r):
    """The arc Gamma_m = circle cap closure(Omega) (eqs. 8, 11) as
    (theta_min, theta_max) with 0 < theta_max - theta_min < 2 pi."""
    angs = boundary_crossings(dom, cx, cy, r)
    uniq = []
    for a in angs:
        if not uniq or a - uniq[-1] > 1e-14:
            uniq.append(a)
    if len(uniq) > 1 and uniq[0] + TWO_PI - uniq[-1] <= 1e-14:
        uniq.pop()
    if not uniq:
        raise CoverError("circle does not cross the boundary but is not floating")
    k = len(uniq)
    ins = []
    for t in range(k):
        a0 = uniq[t]
        a1 = uniq[(t + 1) % k] + (TWO_PI if t + 1 == k else 0.0)
        mid = 0.5 * (a0 + a1)
        ins.append(bool(inside(dom, cx + r * math.cos(mid), cy + r * math.sin(mid))))
    if all(ins):
        raise CoverError("circle touches the boundary without crossing it")
    if not any(ins):
        raise CoverError("circle interface lies outside the domain")
    # maximal cyclic runs of inside intervals
    starts = [t for t in range(k) if ins[t] and not ins[(t - 1) % k]]
    if len(starts) != 1:
        raise CoverError("interface of a perimeter circle has more than one arc")
    s = starts[0]
    e = s
    while ins[(e + 1) % k]:
        e += 1
    theta_min = uniq[s]
    theta_max = uniq[(e + 1) % k]
    if theta_max <= theta_min:
        theta_max += TWO_PI
    return theta_min, theta_max


# ---------------------------------------------------------------------------
# Cover
# ---------------------------------------------------------------------------

@dataclass
class Cover:
    centres: np.ndarray
    radii: np.ndarray
    M: np.ndarray
    Ntheta: np.ndarray
    Nr: np.ndarray
    floating: np.ndarray                 # bool per circle
    arc: np.ndarray                      # (m, 2) theta_min, theta_max (perimeter)
    knot_off: np.ndarray                 # (m+1,) stencil ranges (eq. 9)
    knot_xy: np.ndarray                  # (N, 2)
    knot_theta: np.ndarray               # (N,) local angle on its own circle (eq. 12)
    knot_owner: np.ndarray               # (N,) circle the knot sits on
    knot_boundary: np.ndarray            # (N,) junction knots
    assigned: np.ndarray                 # (N,) circle whose subdomain gives row i, -1 boundary
    row_class: np.ndarray                # (N,) ROW_SPECTRAL / ROW_MC / ROW_BOUNDARY
    rbf_c2: np.ndarray                   # (m,) IMQ shape parameter per perimeter circle
    rowptr: np.ndarray = field(default=None)
    cols: np.ndarray = field(default=None)
    containers: list = field(default=None)   # rule AVERAGED: circles containing each knot

    @property
    def N(self):
        return len(self.knot_xy)

    def stencil(self, m):
        return np.arange(self.knot_off[m], self.knot_off[m + 1])


def build_cover(dom, cov):
    from .cardinal import default_rbf_c2

    centres = np.asarray(cov["centres"], dtype=np.float64)
    radii = np.asarray(cov["radii"], dtype=np.float64)
    M = np.asarray(cov["M"], dtype=np.int64)
    Nth = np.asarray(cov["Ntheta"], dtype=np.int64)
    Nr = np.asarray(cov["Nr"], dtype=np.int64)
    rule = int(cov.get("rule", 0))
    nc = len(radii)
    floating = np.zeros(nc, dtype=bool)
    arc = np.zeros((nc, 2))
    xy, th, own, bnd = [], [], [], []
    knot_off = [0]
    c2 = np.zeros(nc)
    for m in range(nc):
        cx, cy, r = float(centres[m, 0]), float(centres[m, 1]), float(radii[m])
        Mm = int(M[m])
        sd = float(signed_distance(dom, cx, cy))
        if sd - r > 1e-12 * r:
            floating[m] = True
            if Mm % 2 or int(Nth[m]) % 2 or int(Nr[m]) < 1:
                raise CoverError("floating circles need even M and Ntheta and Nr >= 1")
            for j in range(Mm):
                a = TWO_PI * j / Mm
                xy.append((cx + r * math.cos(a), cy + r * math.sin(a)))
                th.append(a)
                own.append(m)
                bnd.append(False)
        else:
            t0, t1 = interface_arc(dom, cx, cy, r)
            arc[m] = (t0, t1)
            span = t1 - t0
            dth = TWO_PI / Mm
            pts = [(t0, math.cos(t0), math.sin(t0), True)]
            grid = []
            for j in range(Mm):
                a = TWO_PI * j / Mm
                off = (a - t0) % TWO_PI
                if 0.25 * dth < off < span - 0.25 * dth:
                    grid.append((t0 + off, math.cos(a), math.sin(a), False))
            grid.sort(key=lambda p: p[0])
            pts += grid
            pts.append((t1, math.cos(t1), math.sin(t1), True))
            for a, ca, sa, isb in pts:
                xy.append((cx + r * ca, cy + r * sa))
                th.append(a)
                own.append(m)
                bnd.append(isb)
            c2v = float(cov.get("rbf_c2", 0.0))
            c2[m] = c2v if c2v > 0.0 else default_rbf_c2(Mm)
        knot_off.append(len(xy))
    knot_xy = np.array(xy, dtype=np.float64).reshape(-1, 2)
    N = len(knot_xy)
    own = np.array(own, dtype=np.int64)
    bnd = np.array(bnd, dtype=bool)

    # row choice (Section 3.2)
    tree = cKDTree(centres)
    rmax = float(radii.max())
    assigned = np.full(N, -1, dtype=np.int64)
    row_class = np.full(N, ROW_BOUNDARY, dtype=np.int64)
    cand_lists = tree.query_ball_point(knot_xy, rmax * (1.0 + 1e-9))
    containers = [[] for _ in range(N)] if rule == RULE_AVERAGED else None
    for i in range(N):
        if bnd[i]:
            continue
        x, y = knot_xy[i]
        best = {True: (-1, 0.0), False: (-1, 0.0)}
        for m in sorted(cand_lists[i]):
            if m == own[i]:
                continue
            dx, dy = x - centres[m, 0], y - centres[m, 1]
            depth = radii[m] - math.sqrt(dx * dx + dy * dy)
            if depth <= 1e-9 * radii[m]:
                continue
            if containers is not None:
                containers[i].append(m)
            key = bool(floating[m]) if rule != 1 else True
            bm, bd = best[key]
            if bm < 0 or depth > bd + 1e-12 * radii[m]:
                best[key] = (m, depth)
        if best[True][0] >= 0:
            m = best[True][0]
        elif best[False][0] >= 0:
            m = best[False][0]
        else:
            raise CoverError(f"knot {i} is not interior to any other subdomain")
        assigned[i] = m
        row_class[i] = ROW_SPECTRAL if floating[m] else ROW_MC

    cov_obj = Cover(centres=centres, radii=radii, M=M, Ntheta=Nth, Nr=Nr,
                    floating=floating, arc=arc,
                    knot_off=np.array(knot_off, dtype=np.int64), knot_xy=knot_xy,
                    knot_theta=np.array(th), knot_owner=own, knot_boundary=bnd,
                    assigned=assigned, row_class=row_class, rbf_c2=c2, containers=containers)
    _csr_pattern(cov_obj)
    return cov_obj


def _csr_pattern(cv):
    """Row i holds the diagonal and, for non-boundary rows, the stencil of the
    chosen circle (eq. 29) -- of every containing circle under rule AVERAGED
    (eq. 38) -- with columns in increasing order."""
    rowptr = [0]
    cols = []
    for i in range(cv.N):
        if cv.row_class[i] == ROW_BOUNDARY:
            c = [i]
        elif cv.containers is not None:
            c = [i]
            for m in cv.containers[i]:
                c += list(range(cv.knot_off[m], cv.knot_off[m + 1]))
            c = sorted(c)
        else:
            m = cv.assigned[i]
            c = sorted([i] + list(range(cv.knot_off[m], cv.knot_off[m + 1])))
        cols.extend(c)
        rowptr.append(len(cols))
    cv.rowptr = np.array(rowptr, dtype=np.int64)
    cv.cols = np.array(cols, dtype=np.int64)


def pair_cover(cv):
    """Rule AVERAGED: a cover whose rows are the pairs (knot i, containing
    circle m), in knot order then circle order, each the row circle m alone
    would give at x_i (eq. 29 for that subdomain) -- stencil columns only, no
    diagonal.  Stencils (knot_off, knot_theta) are those of cv.  Returns the
    cover and the knot of every pair."""
    pk, pm = [], []
    for i in range(cv.N):
        if cv.row_class[i] == ROW_BOUNDARY:
            continue
        for m in cv.containers[i]:
            pk.append(i)
            pm.append(m)
    pk = np.array(pk, dtype=np.int64)
    pm = np.array(pm, dtype=np.int64)
    pc = Cover(centres=cv.centres, radii=cv.radii, M=cv.M, Ntheta=cv.Ntheta, Nr=cv.Nr,
               floating=cv.floating, arc=cv.arc, knot_off=cv.knot_off,
               knot_xy=cv.knot_xy[pk], knot_theta=cv.knot_theta, knot_owner=cv.knot_owner[pk],
               knot_boundary=np.zeros(len(pk), dtype=bool), assigned=pm,
               row_class=np.where(cv.floating[pm], ROW_SPECTRAL, ROW_MC), rbf_c2=cv.rbf_c2)
    rowptr = [0]
    cols = []
    for m in pm:
        cols.extend(range(cv.knot_off[m], cv.knot_off[m + 1]))
        rowptr.append(len(cols))
    pc.rowptr = np.array(rowptr, dtype=np.int64)
    pc.cols = np.array(cols, dtype=np.int64)
    return pc, pk
