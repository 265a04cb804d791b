"""Seeded synthetic workloads shared by the CPU oracle and the HIP library.

This module only draws random numbers and lays out problem descriptions
(domains, circle covers, coefficient-field parameters, Monte Carlo options).
It contains none of the method's arithmetic: no geometry tests, no field
evaluation, no collocation, no sampling of paths.  Both the oracle and the
binding read the plain dictionaries produced here and interpret them with
their own code.

Field descriptors (plain dicts):

* ``{"kind": "const", "value": v}``
* ``{"kind": "sinsum", "base": b, "amp": A, "kx": kx, "ky": ky, "phase": p,
  "clip_nonpos": bool}`` meaning ``base + sum_q A_q sin(2 pi (kx_q x + ky_q y)
  + p_q)``, optionally followed by ``min(., 0)``.
* ``{"kind": "cpoly_re", "alpha": a, "beta": b}`` meaning
  ``Re sum_k (a_k + i b_k) z^k`` with ``z = x + i y``.
* ``{"kind": "derived_f", "u": field}``: the source term that makes ``u`` an
  exact solution of the problem's own operator, in the paper's sign
  convention ``L u + c u + f = 0`` (Section 2, eq. 1).

Coefficient convention (Section 2, eqs. 1-3): the operator is
``a_xx/2 u_xx + a_xy u_xy + a_yy/2 u_yy + b_x u_x + b_y u_y``.  A workload
written as ``a u_xx + a u_yy + b.grad u + c u = f`` is mapped to
``a_xx = a_yy = 2a``, ``a_xy = 0`` and a paper-convention source ``-f``.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi

RULE_FLOAT_FIRST_MAX_DEPTH = 0
RULE_MAX_DEPTH = 1


def const(v):
    return {"kind": "const", "value": float(v)}


def sinsum(base, amp, kx, ky, phase, clip_nonpos=False):
    return {
        "kind": "sinsum",
        "base": float(base),
        "amp": np.asarray(amp, dtype=np.float64),
        "kx": np.asarray(kx, dtype=np.float64),
        "ky": np.asarray(ky, dtype=np.float64),
        "phase": np.asarray(phase, dtype=np.float64),
        "clip_nonpos": bool(clip_nonpos),
    }


def cpoly_re(alpha, beta):
    return {
        "kind": "cpoly_re",
        "alpha": np.asarray(alpha, dtype=np.float64),
        "beta": np.asarray(beta, dtype=np.float64),
    }


def derived_f(u):
    return {"kind": "derived_f", "u": u}


def box(x0=0.0, x1=1.0, y0=0.0, y1=1.0):
    return {"kind": "box", "x0": x0, "x1": x1, "y0": y0, "y1": y1}


def disk(cx, cy, R, holes=()):
    return {"kind": "disk", "cx": cx, "cy": cy, "R": R,
            "holes": [tuple(float(v) for v in h) for h in holes]}


def laplace_problem(domain, g):
    """Laplace: u_xx + u_yy = 0, i.e. a_xx = a_yy = 2, no drift, c = f = 0."""
    return {
        "domain": domain,
        "axx": const(2.0), "axy": const(0.0), "ayy": const(2.0),
        "bx": const(0.0), "by": const(0.0), "c": const(0.0),
        "f": const(0.0), "g": g, "u_exact": g,
    }


def _random_cpoly(rng, degree=4):
    alpha = rng.standard_normal(degree + 1)
    beta = rng.standard_normal(degree + 1)
    return cpoly_re(alpha, beta)


def _wave_vectors(rng, count, kmax):
    choices = [(i, j) for i in range(-kmax, kmax + 1) for j in range(-kmax, kmax + 1)
               if (i, j) != (0, 0)]
    idx = rng.integers(0, len(choices), size=count)
    k = np.array([choices[t] for t in idx], dtype=np.float64)
    return k[:, 0], k[:, 1]


def _random_sinsum(rng, count, std, kmax, clip_nonpos=False):
    amp = rng.normal(0.0, std, size=count)
    kx, ky = _wave_vectors(rng, count, kmax)
    phase = rng.uniform(0.0, TWO_PI, size=count)
    return sinsum(0.0, amp, kx, ky, phase, clip_nonpos)


def lattice_centres(nx, ny, x0=0.0, x1=1.0, y0=0.0, y1=1.0):
    """Centres ((i + 1/2) dx, (j + 1/2) dy), circle index = j * nx + i."""
    xs = x0 + (np.arange(nx) + 0.5) * (x1 - x0) / nx
    ys = y0 + (np.arange(ny) + 0.5) * (y1 - y0) / ny
    X, Y = np.meshgrid(xs, ys)
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def _cover(centres, radii, M, Ntheta, Nr, rbf_c2=0.0, rule=RULE_FLOAT_FIRST_MAX_DEPTH):
    m = len(radii)
    as_i = lambda v: np.broadcast_to(np.asarray(v, dtype=np.int32), (m,)).copy()
    return {
        "centres": np.ascontiguousarray(centres, dtype=np.float64),
        "radii": np.ascontiguousarray(radii, dtype=np.float64),
        "M": as_i(M), "Ntheta": as_i(Ntheta), "Nr": as_i(Nr),
        "rbf_c2": float(rbf_c2), "rule": int(rule),
    }


def mc_opts(paths, h, seed, n_batches=16, step_cap=1 << 20, h_per_circle=None):
    return {
        "paths": int(paths), "h": float(h), "seed": int(seed),
        "n_batches": int(n_batches), "step_cap": int(step_cap),
        "h_per_circle": None if h_per_circle is None
        else np.ascontiguousarray(h_per_circle, dtype=np.float64),
    }


# ---------------------------------------------------------------------------
# The five workloads.  Draw order is part of the definition: each config k
# uses numpy.random.default_rng(k) and draws exactly in the order written.
# ---------------------------------------------------------------------------

def config1(paths=1000, h=1e-3):
    """Laplace on the unit square, 4x4 circles of radius 0.25 at spacing 0.3,
    M = Ntheta = 32, Nr = 12, g = Re p with p a random complex quartic."""
    rng = np.random.default_rng(1)
    g = _random_cpoly(rng, 4)
    prob = laplace_problem(box(), g)
    xs = np.array([0.05, 0.35, 0.65, 0.95])
    X, Y = np.meshgrid(xs, xs)
    centres = np.stack([X.ravel(), Y.ravel()], axis=1)
    cover = _cover(centres, np.full(16, 0.25), 32, 32, 12)
    return {"name": "config1", "problem": prob, "cover": cover,
            "mc": mc_opts(paths, h, seed=1)}


def config2(paths=10000, h=1e-4, n_side=32, radius=0.045):
    """Variable coefficients on the unit square: a = 1 + 0.5 sin(2 pi x) cos(2 pi y),
    b and c random 8-mode sine sums (c clipped to <= 0), manufactured solution
    of 6 random sinusoids; 32x32 circles of radius 0.045, M = Ntheta = 64, Nr = 16."""
    rng = np.random.default_rng(2)
    bx = _random_sinsum(rng, 8, 0.3, 2)
    by = _random_sinsum(rng, 8, 0.3, 2)
    c = _random_sinsum(rng, 8, 0.3, 2, clip_nonpos=True)
    B = rng.standard_normal(6)
    kx, ky = _wave_vectors(rng, 6, 3)
    psi = rng.uniform(0.0, TWO_PI, size=6)
    u = sinsum(0.0, B, kx, ky, psi)
    # 2a = 2 + sin(2 pi x) cos(2 pi y) = 2 + 1/2 sin(2 pi (x + y)) + 1/2 sin(2 pi (x - y))
    two_a = sinsum(2.0, [0.5, 0.5], [1.0, 1.0], [1.0, -1.0], [0.0, 0.0])
    prob = {
        "domain": box(),
        "axx": two_a, "axy": const(0.0), "ayy": two_a,
        "bx": bx, "by": by, "c": c,
        "f": derived_f(u), "g": u, "u_exact": u,
    }
    centres = lattice_centres(n_side, n_side)
    cover = _cover(centres, np.full(len(centres), radius), 64, 64, 16)
    return {"name": "config2", "problem": prob, "cover": cover,
            "mc": mc_opts(paths, h, seed=2)}


def config3(paths=1000, spacing=0.0123, hole=(0.3, 0.0, 0.2)):
    """Unit disk minus an off-centre hole; square lattice of spacing 0.0123 with
    radii spacing * U(0.80, 1.05) and Ntheta drawn from {32,48,64,96,128},
    Nr = Ntheta / 4, M = Ntheta; Laplace with g = Re p; h scaled with r^2."""
    rng = np.random.default_rng(3)
    g = _random_cpoly(rng, 4)
    dom = disk(0.0, 0.0, 1.0, holes=[hole])
    n = int(math.ceil(2.0 / spacing)) + 1
    xs = -1.0 + spacing * np.arange(n)
    X, Y = np.meshgrid(xs, xs)
    centres = np.stack([X.ravel(), Y.ravel()], axis=1)
    radii = spacing * rng.uniform(0.80, 1.05, size=len(centres))
    nth = rng.choice(np.array([32, 48, 64, 96, 128]), size=len(centres))
    # keep circles that meet the open domain (cover condition, Section 2.1 eq. 5)
    d0 = np.hypot(centres[:, 0], centres[:, 1])
    dh = np.hypot(centres[:, 0] - hole[0], centres[:, 1] - hole[1])
    keep = (d0 - radii < 1.0) & (dh + radii > hole[2])
    centres, radii, nth = centres[keep], radii[keep], nth[keep]
    cover = _cover(centres, radii, nth, nth, nth // 4)
    h_pc = 1e-3 * (radii / 0.25) ** 2
    return {"name": "config3", "problem": laplace_problem(dom, g), "cover": cover,
            "mc": mc_opts(paths, 1e-3, seed=3, h_per_circle=h_pc)}


def config4(paths=1000, h=8.1e-6, n_side=64, radius=0.0225):
    """Differentiation workload: Laplace base point on a 64x64 cover, M = Ntheta = 64,
    Nr = 16; loss sum_i (u_i - u_target_i)^2 with u_target = Re p + N(0, 1e-3)."""
    rng = np.random.default_rng(4)
    g = _random_cpoly(rng, 4)
    centres = lattice_centres(n_side, n_side)
    cover = _cover(centres, np.full(len(centres), radius), 64, 64, 16)
    return {"name": "config4", "problem": laplace_problem(box(), g), "cover": cover,
            "mc": mc_opts(paths, h, seed=4), "noise_seed": 40, "noise_std": 1e-3}


def config5(paths=100000, h=1e-5, n_side=128, radius=0.01125):
    """Scale workload: 128x128 cover, M = 64, Ntheta = 48, Nr = 12, Laplace, g = Re p."""
    rng = np.random.default_rng(5)
    g = _random_cpoly(rng, 4)
    centres = lattice_centres(n_side, n_side)
    cover = _cover(centres, np.full(len(centres), radius), 64, 48, 12)
    return {"name": "config5", "problem": laplace_problem(box(), g), "cover": cover,
            "mc": mc_opts(paths, h, seed=5), "noise_seed": 50, "noise_std": 1e-3}


def target_noise(cfg, n):
    """Loss-target noise for the differentiation workloads, drawn after the cover
    is known (n = number of knots)."""
    rng = np.random.default_rng(cfg.get("noise_seed", 0))
    return rng.normal(0.0, cfg.get("noise_std", 1e-3), size=n)


def small_variable(paths=200, h=1e-3, seed=7, n_side=4, radius=0.2, M=16, Ntheta=16, Nr=6):
    """Small variable-coefficient case (config-2 field family) that the oracle
    finishes in about a second; used by the unit and parity tests."""
    rng = np.random.default_rng(seed)
    bx = _random_sinsum(rng, 8, 0.3, 2)
    by = _random_sinsum(rng, 8, 0.3, 2)
    c = _random_sinsum(rng, 8, 0.3, 2, clip_nonpos=True)
    B = rng.standard_normal(6)
    kx, ky = _wave_vectors(rng, 6, 3)
    psi = rng.uniform(0.0, TWO_PI, size=6)
    u = sinsum(0.0, B, kx, ky, psi)
    two_a = sinsum(2.0, [0.5, 0.5], [1.0, 1.0], [1.0, -1.0], [0.0, 0.0])
    axy = sinsum(0.0, [0.2], [1.0], [0.0], [0.3])
    prob = {
        "domain": box(),
        "axx": two_a, "axy": axy, "ayy": two_a,
        "bx": bx, "by": by, "c": c,
        "f": derived_f(u), "g": u, "u_exact": u,
    }
    centres = lattice_centres(n_side, n_side)
    cover = _cover(centres, np.full(len(centres), radius), M, Ntheta, Nr)
    return {"name": "small_variable", "problem": prob, "cover": cover,
            "mc": mc_opts(paths, h, seed=seed)}


def mixed_small(paths=64, h=1e-3, seed=8):
    """Config-3-style uneven resolutions on the small variable-coefficient case:
    the four floating circles of the 4x4 cover get Ntheta = 48, 64, 96, 128
    (collocation sizes 576, 1024, 2304, 4096), the twelve perimeter circles
    Ntheta = 32; M = Ntheta and Nr = Ntheta / 4 throughout."""
    cfg = small_variable(paths=paths, h=h, seed=seed)
    nth = np.full(16, 32, dtype=np.int32)
    nth[[5, 6, 9, 10]] = [48, 64, 96, 128]
    cfg["cover"] = _cover(cfg["cover"]["centres"], cfg["cover"]["radii"], nth, nth, nth // 4)
    cfg["name"] = "mixed_small"
    return cfg


def degenerate(kind, paths=64, h=1e-3, seed=11):
    """Edge covers of the unit square (Laplace, g = Re p with a random cubic):
    "no_floating" -- 2 x 2 circles of radius 0.4, all crossing the boundary
    (no spectral rows, no LU); "one_floating" -- 3 x 3 circles of radius 0.26
    at {0.15, 0.5, 0.85}^2, only the centre one floating (an LU batch of one).
    M = Ntheta = 16, Nr = 6."""
    rng = np.random.default_rng(seed)
    g = _random_cpoly(rng, 3)
    prob = laplace_problem(box(), g)
    if kind == "no_floating":
        xs, r = np.array([0.25, 0.75]), 0.4
    elif kind == "one_floating":
        xs, r = np.array([0.15, 0.5, 0.85]), 0.26
    else:
        raise ValueError(kind)
    X, Y = np.meshgrid(xs, xs)
    centres = np.stack([X.ravel(), Y.ravel()], axis=1)
    cover = _cover(centres, np.full(len(centres), r), 16, 16, 6)
    return {"name": kind, "problem": prob, "cover": cover, "mc": mc_opts(paths, h, seed=seed)}


def eq46():
    """The manufactured solution of Section 4 (eq. 46), evaluated by the library."""
    return {"kind": "eq46"}


def paper_poisson(half=50.0, paths=5000, h=0.015, seed=46, rule=RULE_FLOAT_FIRST_MAX_DEPTH, scheme=0):
    """Section 4's test problem: Poisson's equation with the exact solution of
    eq. 46 and Dirichlet data equal to it, on the square [-half, half]^2.
    Circles on a square lattice of spacing 10 (100 circles at half = 50, as in
    Table 1; Figure 5's exact layout is not available), radii drawn uniformly
    in [8.55, 9.43], 44 knots and 44 x 22 collocation nodes per circle (n = 968),
    c^2 = 1.5, paths per perimeter knot and h as in Section 4.  ``rule`` picks
    the row choice (2: averaged rows) and ``scheme`` the integrator (0 plain
    Euler, 1 boundary-shifted Gobet-Menozzi; the paper's variance reduction is
    not included)."""
    rng = np.random.default_rng(seed)
    n_side = int(round(2.0 * half / 10.0))
    centres = lattice_centres(n_side, n_side, -half, half, -half, half)
    radii = rng.uniform(8.55, 9.43, size=len(centres))
    u = eq46()
    prob = {
        "domain": box(-half, half, -half, half),
        "axx": const(2.0), "axy": const(0.0), "ayy": const(2.0),
        "bx": const(0.0), "by": const(0.0), "c": const(0.0),
        "f": derived_f(u), "g": u, "u_exact": u,
    }
    cover = _cover(centres, radii, 44, 44, 22, rbf_c2=1.5, rule=rule)
    mc = mc_opts(paths, h, seed=seed)
    mc["scheme"] = int(scheme)
    return {"name": f"paper_poisson_{int(half)}", "problem": prob, "cover": cover, "mc": mc}


def paper_poisson_as_run(half=50.0):
    """Section 4's problem with the paper's row choice (averaged rows, which
    Table 1's density points to) and integrator (boundary-shifted Euler)."""
    return paper_poisson(half=half, rule=2, scheme=1)


CONFIGS = {
    "config1": config1, "config2": config2, "config3": config3,
    "config4": config4, "config5": config5,
    "paper50": paper_poisson,
    "paper50_gm": paper_poisson_as_run,
}
