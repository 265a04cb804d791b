"""The explicit interfacial system C u = r (Section 2.3, eqs. 28-30), assembled
from floating rows (local spectral solves, eqs. 31-35) and perimeter rows
(Monte Carlo, eqs. 29-30), its direct solve and the diagnostics of Table 1.

Boundary (junction) knots carry the Dirichlet data: C_ii = 1, r_i = g(x_i).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fields, geometry, montecarlo, spectral
from .geometry import ROW_BOUNDARY, ROW_MC, ROW_SPECTRAL


@dataclass
class System:
    cover: geometry.Cover
    val: np.ndarray        # CSR values aligned with cover.rowptr / cover.cols
    b: np.ndarray
    se: np.ndarray         # per-entry Monte Carlo standard error (0 if exact)
    se_b: np.ndarray
    path_steps: int

    def matrix(self):
        N = self.cover.N
        return sp.csr_matrix((self.val, self.cover.cols, self.cover.rowptr), shape=(N, N))


def _put_row(cover, val, se, i, m, entries, entries_se=None):
    lo, hi = cover.rowptr[i], cover.rowptr[i + 1]
    cols = cover.cols[lo:hi]
    off = cover.knot_off[m]
    for t, c in enumerate(cols):
        if c == i:
            val[lo + t] = 1.0
        else:
            val[lo + t] = entries[c - off]
            if entries_se is not None:
                se[lo + t] = entries_se[c - off]


def assemble(problem, cover, mc, samples=None, with_mc=True, circles=None):
    """Assemble C (CSR) and r.  ``samples`` optionally maps floating circle index
    to its seven node samples; otherwise the fields are sampled at the nodes.
    ``circles`` restricts the floating circles processed (others left zero)."""
    if cover.containers is not None:
        return _assemble_averaged(problem, cover, mc, samples, with_mc, circles)
    N = cover.N
    val = np.zeros(len(cover.cols))
    se = np.zeros(len(cover.cols))
    b = np.zeros(N)
    se_b = np.zeros(N)
    float_ids = np.nonzero(cover.floating)[0] if circles is None else np.asarray(circles)
    for m in float_ids:
        s = None if samples is None else samples[m]
        knots, Crows, rv = spectral.floating_rows(problem, cover, m, s)
        for t, i in enumerate(knots):
            _put_row(cover, val, se, i, m, Crows[t])
            b[i] = rv[t]
    steps = 0
    if with_mc:
        knots, rows, ses, r, se_r, steps = montecarlo.mc_rows(problem, cover, mc)
        for t, i in enumerate(knots):
            _put_row(cover, val, se, i, cover.assigned[i], rows[t], ses[t])
            b[i] = r[t]
            se_b[i] = se_r[t]
    bnd = np.nonzero(cover.row_class == ROW_BOUNDARY)[0]
    for i in bnd:
        val[cover.rowptr[i]] = 1.0
    if len(bnd):
        b[bnd] = fields.value(problem["g"], cover.knot_xy[bnd, 0], cover.knot_xy[bnd, 1], problem)
    return System(cover, val, b, se, se_b, steps)


def solve(system, rhs=None, transpose=False):
    """u = C^-1 r by sparse LU (SuperLU)."""
    A = system.matrix()
    if transpose:
        A = A.T
    lu = spla.splu(sp.csc_matrix(A))
    return lu.solve(system.b if rhs is None else rhs)


def diagnostics(system, u=None, u_exact=None):
    """N, nnz, sparsity, max off-diagonal entry, spectral radius of C - I
    (dense, for small N), RMS error against an exact solution."""
    A = system.matrix()
    N = A.shape[0]
    out = {"N": N, "nnz": A.nnz, "sparsity": A.nnz / N / N}
    off = A - sp.diags(A.diagonal())
    out["max_offdiag"] = float(off.max()) if off.nnz else 0.0
    if N <= 4000:
        ev = np.linalg.eigvals((A - sp.eye(N)).toarray())
        out["rho_C_minus_I"] = float(np.max(np.abs(ev)))
    if u is not None and u_exact is not None:
        out["rms_error"] = float(np.sqrt(np.mean((u - u_exact) ** 2)))
    return out


def _assemble_averaged(problem, cover, mc, samples, with_mc, circles):
    """Rule AVERAGED (eqs. 38-39): every pair (knot i, circle m containing it)
    is the row circle m alone gives at x_i -- spectral for a floating m, Monte
    Carlo (with the pair's own random stream: the pair index is the knot word
    of the Philox counter) for a perimeter m; row i is C_ii = #Pi_i and the
    pairs' stencil entries side by side, r_i the sum of the pairs' r in pair
    order, standard errors added in quadrature."""
    pc, pknot = geometry.pair_cover(cover)
    P = pc.N
    prow = [None] * P          # stencil entries of each pair
    pse = [None] * P
    pb = np.zeros(P)
    pse_b = np.zeros(P)
    float_ids = np.nonzero(cover.floating)[0] if circles is None else np.asarray(circles)
    for m in float_ids:
        s = None if samples is None else samples[m]
        knots, Crows, rv = spectral.floating_rows(problem, pc, m, s)
        for t, p in enumerate(knots):
            prow[p] = Crows[t]
            pb[p] = rv[t]
    steps = 0
    if with_mc:
        knots, rows, ses, r, se_r, steps = montecarlo.mc_rows(problem, pc, mc)
        for t, p in enumerate(knots):
            prow[p] = rows[t]
            pse[p] = ses[t]
            pb[p] = r[t]
            pse_b[p] = se_r[t]
    N = cover.N
    val = np.zeros(len(cover.cols))
    se = np.zeros(len(cover.cols))
    b = np.zeros(N)
    se_b2 = np.zeros(N)
    for p in range(P):
        i, m = int(pknot[p]), int(pc.assigned[p])
        lo, hi = cover.rowptr[i], cover.rowptr[i + 1]
        cols = cover.cols[lo:hi]
        off = cover.knot_off[m]
        seg = lo + int(np.searchsorted(cols, off))
        if prow[p] is not None:
            val[seg:seg + len(prow[p])] = prow[p]
            if pse[p] is not None:
                se[seg:seg + len(pse[p])] = pse[p]
        b[i] += pb[p]
        se_b2[i] += pse_b[p] ** 2
    for i in range(N):
        if cover.row_class[i] == ROW_BOUNDARY:
            continue
        lo, hi = cover.rowptr[i], cover.rowptr[i + 1]
        d = lo + int(np.searchsorted(cover.cols[lo:hi], i))
        val[d] = float(len(cover.containers[i]))
    bnd = np.nonzero(cover.row_class == ROW_BOUNDARY)[0]
    for i in bnd:
        val[cover.rowptr[i]] = 1.0
    if len(bnd):
        b[bnd] = fields.value(problem["g"], cover.knot_xy[bnd, 0], cover.knot_xy[bnd, 1], problem)
    return System(cover, val, b, se, np.sqrt(se_b2), steps)
