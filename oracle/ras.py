"""One-level restricted additive Schwarz preconditioner and right-preconditioned
restarted GMRES for C u = r (Section 4, eqs. 42-45).  Test infrastructure:
only the tests, the smoke check and the CPU baseline use this module.

Readings taken where the paper leaves details open:

* Non-overlapping partition: the paper partitions the graph of C with METIS.
  Here the circles are split geometrically: sorted by centre x (stable, ties
  by index) into ``px`` slabs of near-equal circle counts, slab s taking
  sorted positions [s n / px, (s + 1) n / px); each slab sorted by centre y
  the same way into ``py`` parts.  A knot belongs to the part of the circle
  it lies on.  Empty parts are dropped.
* Overlap: omega_p is the knots of part p plus every knot adjacent to one of
  them in the graph of C, taken symmetric (C_ij or C_ji structurally
  nonzero), one layer.
* D_p (eq. 43) weights knot i by 1 / #{q : x_i in omega_q}.
* GMRES: restarted every ``restart`` iterations, Arnoldi with modified
  Gram-Schmidt, Givens rotations on the Hessenberg matrix, zero initial
  guess, stops when the preconditioned system's residual estimate
  |g_{j+1}| <= rtol |r| (equal to the true residual |r - C u| in exact
  arithmetic, since the preconditioner is on the right).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def partition(cover, px, py):
    """Part of every knot (array [N]) and the number of non-empty parts."""
    n = len(cover.radii)
    cx = np.asarray(cover.centres)[:, 0]
    cy = np.asarray(cover.centres)[:, 1]
    part_of_circle = np.empty(n, dtype=np.int64)
    by_x = np.argsort(cx, kind="stable")
    for s in range(px):
        slab = by_x[s * n // px:(s + 1) * n // px]
        by_y = slab[np.argsort(cy[slab], kind="stable")]
        k = len(by_y)
        for t in range(py):
            part_of_circle[by_y[t * k // py:(t + 1) * k // py]] = s * py + t
    used = np.unique(part_of_circle)
    renum = np.full(px * py, -1, dtype=np.int64)
    renum[used] = np.arange(len(used))
    return renum[part_of_circle[np.asarray(cover.knot_owner)]], len(used)


def subdomains(cover, px, py):
    """omega_p (sorted knot lists, the overlapping partition of eq. 42) and the
    diagonal of D_p for each (eq. 43)."""
    part, P = partition(cover, px, py)
    N = cover.N
    A = sp.csr_matrix((np.ones(len(cover.cols)), cover.cols, cover.rowptr), shape=(N, N))
    G = ((A + A.T) != 0).tocsr()
    omegas = []
    for p in range(P):
        own = np.nonzero(part == p)[0]
        nb = G[own].indices
        omegas.append(np.union1d(own, nb))
    mult = np.zeros(N)
    for w in omegas:
        mult[w] += 1.0
    D = [1.0 / mult[w] for w in omegas]
    return omegas, D


class RAS:
    """M_RAS^-1 = sum_p R_p^T D_p C_p^-1 R_p (eq. 44), C_p = R_p C R_p^T (eq. 42),
    each C_p factorised by LU with partial pivoting."""

    def __init__(self, C, cover, px, py):
        self.omegas, self.D = subdomains(cover, px, py)
        C = sp.csr_matrix(C)
        self.lu = [sla.lu_factor(C[w][:, w].toarray()) for w in self.omegas]
        self.N = C.shape[0]

    def apply(self, x):
        y = np.zeros(self.N)
        for w, d, f in zip(self.omegas, self.D, self.lu):
            y[w] += d * sla.lu_solve(f, x[w])
        return y


def gmres(C, b, M=None, rtol=1e-10, restart=30, max_iter=2000):
    """Right-preconditioned restarted GMRES (eq. 45): solves C M^-1 t = b and
    returns u = M^-1 t, the iteration count and the final relative residual
    estimate.  M is an object with ``apply`` or None."""
    C = sp.csr_matrix(C)
    N = C.shape[0]
    prec = (lambda v: M.apply(v)) if M is not None else (lambda v: v.copy())
    u = np.zeros(N)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return u, 0, 0.0
    it = 0
    rel = 1.0
    while it < max_iter:
        r = b - C @ u
        beta = float(np.linalg.norm(r))
        rel = beta / bnorm
        if rel <= rtol:
            break
        V = np.zeros((restart + 1, N))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(restart):
            w = C @ prec(V[j])
            for i in range(j + 1):           # modified Gram-Schmidt
                H[i, j] = float(w @ V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):               # earlier rotations on the new column
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            rel = abs(g[j + 1]) / bnorm
            if rel <= rtol or it >= max_iter:
                break
        y = sla.solve_triangular(H[:k, :k], g[:k])
        u = u + prec(V[:k].T @ y)
        if rel <= rtol:
            break
    return u, it, rel
