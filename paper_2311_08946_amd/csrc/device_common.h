// Device-side problem description: coefficient fields of eq. 1 and the domain,
// evaluated at collocation nodes and along Monte Carlo paths.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "pdd.h"

namespace pdd {

struct DevField {
  int32_t kind, n, clip, pad;
  double base;
  double a[PDD_MAX_TERMS], b[PDD_MAX_TERMS], c[PDD_MAX_TERMS], d[PDD_MAX_TERMS];
};

enum { F_AXX = 0, F_AXY, F_AYY, F_BX, F_BY, F_C, F_F, F_G, F_U, F_COUNT };

struct DevProblem {
  pdd_domain dom;
  DevField fld[F_COUNT];
  int32_t const_coef;        // every coefficient and f is PDD_FIELD_CONST
  int32_t pad;
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

__device__ __forceinline__ double field_plain(const DevField& F, double x, double y) {
  if (F.kind == PDD_FIELD_CONST) return F.base;
  if (F.kind == PDD_FIELD_SINSUM) return sinsum_value(F, x, y);
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
