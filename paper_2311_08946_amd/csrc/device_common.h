// Device-side problem description: coefficient fields of eq. 1 and the domain,
// evaluated at collocation nodes and along Monte Carlo paths.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "pdd.h"

namespace pdd {

// Largest |wave number| of a sine-sum term that the Monte Carlo kernels
// evaluate from a per-lane table of powers instead of a sine per term.
constexpr int kWaveMax = 4;

struct DevField {
  int32_t kind, n, clip;
  int32_t wave;          // SINSUM with integer wave numbers, |b|, |c| <= kWaveMax
  double base;
  double a[PDD_MAX_TERMS], b[PDD_MAX_TERMS], c[PDD_MAX_TERMS], d[PDD_MAX_TERMS];
  // with `wave`: term q is Im(w_q e^{2 pi i (b_q x + c_q y)}), w_q = a_q e^{i d_q}
  // = (wr_q, wi_q); ix, iy = |b_q|, |c_q|; sx, sy = their signs (+1 for 0)
  int32_t ix[PDD_MAX_TERMS], iy[PDD_MAX_TERMS];
  double sx[PDD_MAX_TERMS], sy[PDD_MAX_TERMS], wr[PDD_MAX_TERMS], wi[PDD_MAX_TERMS];
};

enum { F_AXX = 0, F_AXY, F_AYY, F_BX, F_BY, F_C, F_F, F_G, F_U, F_COUNT };

struct DevProblem {
  pdd_domain dom;
  DevField fld[F_COUNT];
  int32_t const_coef;        // every coefficient and f is PDD_FIELD_CONST
  int32_t wave_all;          // every coefficient and f is CONST or a `wave` sine sum (f
                             // possibly derived from a `wave` u), and not all are CONST
  double k[7];               // their values when const_coef
};

constexpr double kTwoPiD = 6.283185307179586476925286766559;

__device__ __forceinline__ double sinsum_value(const DevField& F, double x, double y) {
  double v = F.base;
  for (int q = 0; q < F.n; ++q) v += F.a[q] * sin(kTwoPiD * (F.b[q] * x + F.c[q] * y) + F.d[q]);
  if (F.clip) v = fmin(v, 0.0);
  return v;
}

// p(z) = sum_k (a_k + i b_k) z^k by Horner, with p' and p''.
__device__ __forceinline__ void cpoly_jet(const DevField& F, double x, double y, double& pr,
                                          double& pi, double& d1r, double& d1i, double& d2r,
                                          double& d2i) {
  pr = pi = d1r = d1i = d2r = d2i = 0.0;
  for (int k = F.n - 1; k >= 0; --k) {
    // p'' <- p'' z + 2 p'; p' <- p' z + p; p <- p z + coef  (Horner for derivatives)
    double t2r = d2r * x - d2i * y + 2.0 * d1r;
    double t2i = d2r * y + d2i * x + 2.0 * d1i;
    double t1r = d1r * x - d1i * y + pr;
    double t1i = d1r * y + d1i * x + pi;
    double t0r = pr * x - pi * y + F.a[k];
    double t0i = pr * y + pi * x + F.b[k];
    d2r = t2r; d2i = t2i; d1r = t1r; d1i = t1i; pr = t0r; pi = t0i;
  }
}

// The manufactured solution of Section 4 (eq. 46) and its derivatives up to
// second order: u = 3 + sin(rho)/3 + tanh(s)/3 with rho = sqrt(1 + x^2/100 +
// y^2/50) and s = sin(3x/25 + y/20) + sin(x/20 - 3y/25).
__device__ __forceinline__ void eq46_jet(double x, double y, double* j) {
  const double rho = sqrt(1.0 + x * x / 100.0 + y * y / 50.0);
  const double rx = x / (100.0 * rho), ry = y / (50.0 * rho);
  const double r3 = rho * rho * rho;
  const double rxx = 1.0 / (100.0 * rho) - x * x / (10000.0 * r3);
  const double ryy = 1.0 / (50.0 * rho) - y * y / (2500.0 * r3);
  const double rxy = -x * y / (5000.0 * r3);
  double sr, cr;
  sincos(rho, &sr, &cr);
  const double al = 3.0 * x / 25.0 + y / 20.0, be = x / 20.0 - 3.0 * y / 25.0;
  double sa, ca, sb, cb;
  sincos(al, &sa, &ca);
  sincos(be, &sb, &cb);
  const double s = sa + sb;
  const double sx = 0.12 * ca + 0.05 * cb, sy = 0.05 * ca - 0.12 * cb;
  const double sxx = -0.0144 * sa - 0.0025 * sb, syy = -0.0025 * sa - 0.0144 * sb;
  const double sxy = -0.006 * sa + 0.006 * sb;
  const double T = tanh(s), T1 = 1.0 - T * T, T2 = -2.0 * T * T1;
  const double third = 1.0 / 3.0;
  j[0] = 3.0 + third * (sr + T);
  j[1] = third * (cr * rx + T1 * sx);
  j[2] = third * (cr * ry + T1 * sy);
  j[3] = third * (-sr * rx * rx + cr * rxx + T2 * sx * sx + T1 * sxx);
  j[4] = third * (-sr * rx * ry + cr * rxy + T2 * sx * sy + T1 * sxy);
  j[5] = third * (-sr * ry * ry + cr * ryy + T2 * sy * sy + T1 * syy);
}

__device__ __forceinline__ double field_plain(const DevField& F, double x, double y) {
  if (F.kind == PDD_FIELD_CONST) return F.base;
  if (F.kind == PDD_FIELD_SINSUM) return sinsum_value(F, x, y);
  if (F.kind == PDD_FIELD_EQ46) {
    double j[6];
    eq46_jet(x, y, j);
    return j[0];
  }
  double pr, pi, a, b, c, d;
  cpoly_jet(F, x, y, pr, pi, a, b, c, d);
  return pr;
}

// (u, u_x, u_y, u_xx, u_xy, u_yy) of a manufactured solution.
__device__ __forceinline__ void field_jet(const DevField& F, double x, double y, double* j) {
  if (F.kind == PDD_FIELD_SINSUM) {
    double u = F.base, ux = 0, uy = 0, uxx = 0, uxy = 0, uyy = 0;
    for (int q = 0; q < F.n; ++q) {
      double s, c;
      sincos(kTwoPiD * (F.b[q] * x + F.c[q] * y) + F.d[q], &s, &c);
      double kx = kTwoPiD * F.b[q], ky = kTwoPiD * F.c[q], A = F.a[q];
      u += A * s;
      ux += A * kx * c;
      uy += A * ky * c;
      uxx -= A * kx * kx * s;
      uxy -= A * kx * ky * s;
      uyy -= A * ky * ky * s;
    }
    j[0] = u; j[1] = ux; j[2] = uy; j[3] = uxx; j[4] = uxy; j[5] = uyy;
  } else if (F.kind == PDD_FIELD_EQ46) {
    eq46_jet(x, y, j);
  } else if (F.kind == PDD_FIELD_CPOLY_RE) {
    double pr, pi, d1r, d1i, d2r, d2i;
    cpoly_jet(F, x, y, pr, pi, d1r, d1i, d2r, d2i);
    j[0] = pr; j[1] = d1r; j[2] = -d1i; j[3] = d2r; j[4] = -d2i; j[5] = -d2r;
  } else {
    j[0] = F.base; j[1] = j[2] = j[3] = j[4] = j[5] = 0.0;
  }
}

// The seven coefficients (axx, axy, ayy, bx, by, c, f) of eq. 1 at (x, y).
__device__ __forceinline__ void coefficients_at(const DevProblem& P, double x, double y, double* co) {
  if (P.const_coef) {
    for (int t = 0; t < 7; ++t) co[t] = P.k[t];
    return;
  }
  for (int t = 0; t < 6; ++t) co[t] = field_plain(P.fld[t], x, y);
  const DevField& F = P.fld[F_F];
  if (F.kind == PDD_FIELD_DERIVED_F) {
    double j[6];
    field_jet(P.fld[F_U], x, y, j);
    co[6] = -(0.5 * co[0] * j[3] + co[1] * j[4] + 0.5 * co[2] * j[5] + co[3] * j[1] +
              co[4] * j[2] + co[5] * j[0]);
  } else {
    co[6] = field_plain(F, x, y);
  }
}

// Per-lane table of the powers E^k and F^k, k = 0 .. kWaveMax, of
// E = e^{2 pi i x} and F = e^{2 pi i y} (E^k at p[k stride], F^k at
// p[(kWaveMax + 1 + k) stride], each as (re, im)), so that a sine-sum term
// with integer wave numbers costs a complex product instead of a sine:
// a sin(2 pi (b x + c y) + d) = Im(a e^{i d} E^b F^c), E^-k = conj(E^k).
struct WaveTab {
  double2* p;   // this lane's first entry (LDS)
  int stride;   // entries between powers
};

__device__ __forceinline__ void wave_fill(const WaveTab& t, double x, double y) {
  double es, ec, fs, fc;
  sincospi(2.0 * x, &es, &ec);
  sincospi(2.0 * y, &fs, &fc);
  double er = 1.0, ei = 0.0, fr = 1.0, fi = 0.0;
#pragma unroll
  for (int k = 0; k <= kWaveMax; ++k) {
    t.p[k * t.stride] = double2{er, ei};
    t.p[(kWaveMax + 1 + k) * t.stride] = double2{fr, fi};
    const double er1 = er * ec - ei * es, ei1 = er * es + ei * ec;
    const double fr1 = fr * fc - fi * fs, fi1 = fr * fs + fi * fc;
    er = er1; ei = ei1; fr = fr1; fi = fi1;
  }
}

// e^{2 pi i (b_q x + c_q y)} of term q from the table
__device__ __forceinline__ void wave_term(const DevField& F, int q, const WaveTab& t, double& zr, double& zi) {
  const double2 e = t.p[F.ix[q] * t.stride];
  const double2 f = t.p[(kWaveMax + 1 + F.iy[q]) * t.stride];
  const double ey = F.sx[q] * e.y, fy = F.sy[q] * f.y;
  zr = e.x * f.x - ey * fy;
  zi = e.x * fy + ey * f.x;
}

__device__ __forceinline__ double sinsum_tab(const DevField& F, const WaveTab& t) {
  double v = F.base;
  for (int q = 0; q < F.n; ++q) {
    double zr, zi;
    wave_term(F, q, t, zr, zi);
    v += F.wr[q] * zi + F.wi[q] * zr;
  }
  if (F.clip) v = fmin(v, 0.0);
  return v;
}

// field_jet of a `wave` sine sum from the table
__device__ __forceinline__ void sinsum_jet_tab(const DevField& F, const WaveTab& t, double* j) {
  double u = F.base, ux = 0, uy = 0, uxx = 0, uxy = 0, uyy = 0;
  for (int q = 0; q < F.n; ++q) {
    double zr, zi;
    wave_term(F, q, t, zr, zi);
    const double as = F.wr[q] * zi + F.wi[q] * zr;   // a sin(theta)
    const double ac = F.wr[q] * zr - F.wi[q] * zi;   // a cos(theta)
    const double kx = kTwoPiD * F.b[q], ky = kTwoPiD * F.c[q];
    u += as;
    ux += kx * ac;
    uy += ky * ac;
    uxx -= kx * kx * as;
    uxy -= kx * ky * as;
    uyy -= ky * ky * as;
  }
  j[0] = u; j[1] = ux; j[2] = uy; j[3] = uxx; j[4] = uxy; j[5] = uyy;
}

// coefficients_at for the Monte Carlo kernels when `wave_all` holds: the
// table is filled for (x, y) and every sine sum read from it.
__device__ __forceinline__ void coefficients_wave(const DevProblem& P, double x, double y, double* co,
                                                  const WaveTab& t) {
  wave_fill(t, x, y);
  for (int k = 0; k < 6; ++k) {
    const DevField& F = P.fld[k];
    co[k] = F.kind == PDD_FIELD_CONST ? F.base : sinsum_tab(F, t);
  }
  const DevField& F = P.fld[F_F];
  if (F.kind == PDD_FIELD_DERIVED_F) {
    double j[6];
    sinsum_jet_tab(P.fld[F_U], t, j);
    co[6] = -(0.5 * co[0] * j[3] + co[1] * j[4] + 0.5 * co[2] * j[5] + co[3] * j[1] +
              co[4] * j[2] + co[5] * j[0]);
  } else {
    co[6] = F.kind == PDD_FIELD_CONST ? F.base : sinsum_tab(F, t);
  }
}

__device__ __forceinline__ double boundary_value(const DevProblem& P, double x, double y) {
  return field_plain(P.fld[F_G], x, y);
}

__device__ __forceinline__ bool in_domain(const pdd_domain& d, double x, double y) {
  if (d.kind == PDD_DOMAIN_BOX) return x > d.x0 && x < d.x1 && y > d.y0 && y < d.y1;
  double ex = x - d.cx, ey = y - d.cy;
  if (!(ex * ex + ey * ey < d.R * d.R)) return false;
  for (int h = 0; h < d.n_holes; ++h) {
    double hx = x - d.holes[h][0], hy = y - d.holes[h][1], hr = d.holes[h][2];
    if (hx * hx + hy * hy <= hr * hr) return false;
  }
  return true;
}

}  // namespace pdd
