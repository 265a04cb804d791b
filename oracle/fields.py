"""Coefficient fields of the model problem (Section 2, eqs. 1-3).

The problem is  L u + c u + f = 0  in Omega, u = g on the boundary, with
L = a_xx/2 d_xx + a_xy d_xy + a_yy/2 d_yy + b_x d_x + b_y d_y.
Fields are described by the plain dicts of the ``workloads`` module; this
module evaluates them (and the derivatives of manufactured solutions) with
NumPy in float64.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def _sinsum_parts(fd, x, y):
    """Phases 2 pi (kx x + ky y) + p for every term, shape (npts, nterms)."""
    x = np.asarray(x, dtype=np.float64)[..., None]
    y = np.asarray(y, dtype=np.float64)[..., None]
    return TWO_PI * (fd["kx"] * x + fd["ky"] * y) + fd["phase"]


def _cpoly(fd, z):
    """p(z) = sum_k (alpha_k + i beta_k) z^k and its first two derivatives."""
    coef = fd["alpha"] + 1j * fd["beta"]
    p = np.zeros_like(z)
    dp = np.zeros_like(z)
    d2p = np.zeros_like(z)
    for k, a in enumerate(coef):
        p = p + a * z ** k
        if k >= 1:
            dp = dp + k * a * z ** (k - 1)
        if k >= 2:
            d2p = d2p + k * (k - 1) * a * z ** (k - 2)
    return p, dp, d2p


def _eq46(x, y):
    """The manufactured solution of Section 4, eq. 46, with its first and
    second derivatives (chain rule on rho = sqrt(1 + x^2/100 + y^2/50) and on
    s = sin(3x/25 + y/20) + sin(x/20 - 3y/25)):
    u = 3 + sin(rho)/3 + tanh(s)/3."""
    q = 1.0 + x * x / 100.0 + y * y / 50.0
    rho = np.sqrt(q)
    # derivatives of q, then of rho = q^(1/2)
    qx, qy, qxx, qyy = x / 50.0, y / 25.0, 1.0 / 50.0, 1.0 / 25.0
    rx, ry = qx / (2.0 * rho), qy / (2.0 * rho)
    rxx = qxx / (2.0 * rho) - qx * qx / (4.0 * rho ** 3)
    ryy = qyy / (2.0 * rho) - qy * qy / (4.0 * rho ** 3)
    rxy = -qx * qy / (4.0 * rho ** 3)
    # s and its derivatives: d(alpha) = (3/25, 1/20), d(beta) = (1/20, -3/25)
    a1, a2 = 3.0 / 25.0, 1.0 / 20.0
    b1, b2 = 1.0 / 20.0, -3.0 / 25.0
    alpha = a1 * x + a2 * y
    beta = b1 * x + b2 * y
    s = np.sin(alpha) + np.sin(beta)
    sx = a1 * np.cos(alpha) + b1 * np.cos(beta)
    sy = a2 * np.cos(alpha) + b2 * np.cos(beta)
    sxx = -a1 * a1 * np.sin(alpha) - b1 * b1 * np.sin(beta)
    syy = -a2 * a2 * np.sin(alpha) - b2 * b2 * np.sin(beta)
    sxy = -a1 * a2 * np.sin(alpha) - b1 * b2 * np.sin(beta)
    t = np.tanh(s)
    dt = 1.0 - t * t              # tanh'
    d2t = -2.0 * t * dt           # tanh''
    u = 3.0 + (np.sin(rho) + t) / 3.0
    ux = (np.cos(rho) * rx + dt * sx) / 3.0
    uy = (np.cos(rho) * ry + dt * sy) / 3.0
    uxx = (-np.sin(rho) * rx * rx + np.cos(rho) * rxx + d2t * sx * sx + dt * sxx) / 3.0
    uxy = (-np.sin(rho) * rx * ry + np.cos(rho) * rxy + d2t * sx * sy + dt * sxy) / 3.0
    uyy = (-np.sin(rho) * ry * ry + np.cos(rho) * ryy + d2t * sy * sy + dt * syy) / 3.0
    return u, ux, uy, uxx, uxy, uyy


def value(fd, x, y, problem=None):
    """Field value at points (x, y)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    kind = fd["kind"]
    if kind == "const":
        return np.full(np.broadcast(x, y).shape, fd["value"])
    if kind == "sinsum":
        v = fd["base"] + np.sum(fd["amp"] * np.sin(_sinsum_parts(fd, x, y)), axis=-1)
        if fd["clip_nonpos"]:
            v = np.minimum(v, 0.0)
        return v
    if kind == "cpoly_re":
        p, _, _ = _cpoly(fd, x + 1j * y)
        return p.real
    if kind == "eq46":
        return _eq46(x, y)[0]
    if kind == "derived_f":
        if problem is None:
            raise ValueError("derived_f needs the problem's coefficient fields")
        return derived_source(problem, fd["u"], x, y)
    raise ValueError(f"unknown field kind {kind}")


def jet(fd, x, y):
    """(u, u_x, u_y, u_xx, u_xy, u_yy) of a manufactured solution."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    kind = fd["kind"]
    if kind == "sinsum":
        if fd["clip_nonpos"]:
            raise ValueError("a clipped field has no smooth jet")
        ph = _sinsum_parts(fd, x, y)
        s, c = np.sin(ph), np.cos(ph)
        A, kx, ky = fd["amp"], TWO_PI * fd["kx"], TWO_PI * fd["ky"]
        u = fd["base"] + np.sum(A * s, axis=-1)
        ux = np.sum(A * kx * c, axis=-1)
        uy = np.sum(A * ky * c, axis=-1)
        uxx = -np.sum(A * kx * kx * s, axis=-1)
        uxy = -np.sum(A * kx * ky * s, axis=-1)
        uyy = -np.sum(A * ky * ky * s, axis=-1)
        return u, ux, uy, uxx, uxy, uyy
    if kind == "cpoly_re":
        # Re p is harmonic; with p' = dp/dz: u_x = Re p', u_y = -Im p',
        # u_xx = Re p'', u_xy = -Im p'', u_yy = -Re p''.
        p, dp, d2p = _cpoly(fd, x + 1j * y)
        return p.real, dp.real, -dp.imag, d2p.real, -d2p.imag, -d2p.real
    if kind == "eq46":
        return _eq46(x, y)
    if kind == "const":
        z = np.zeros(np.broadcast(x, y).shape)
        return z + fd["value"], z, z, z, z, z
    raise ValueError(f"field kind {kind} has no jet")


def derived_source(problem, ufd, x, y):
    """f such that u solves L u + c u + f = 0 (eq. 1): f = -(L u + c u)."""
    u, ux, uy, uxx, uxy, uyy = jet(ufd, x, y)
    axx = value(problem["axx"], x, y)
    axy = value(problem["axy"], x, y)
    ayy = value(problem["ayy"], x, y)
    bx = value(problem["bx"], x, y)
    by = value(problem["by"], x, y)
    c = value(problem["c"], x, y)
    Lu = 0.5 * axx * uxx + axy * uxy + 0.5 * ayy * uyy + bx * ux + by * uy
    return -(Lu + c * u)


def coefficients(problem, x, y):
    """All seven coefficient samples of eq. 1 at the given points."""
    return {name: value(problem[name], x, y, problem)
            for name in ("axx", "axy", "ayy", "bx", "by", "c", "f")}


def sigma(axx, axy, ayy):
    """Lower Cholesky factor of [[a_xx, a_xy], [a_xy, a_yy]] (eq. 3)."""
    s11 = np.sqrt(axx)
    s21 = axy / s11
    s22 = np.sqrt(ayy - s21 * s21)
    return s11, s21, s22
