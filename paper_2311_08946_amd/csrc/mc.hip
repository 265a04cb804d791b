// Perimeter rows of C and r on gfx950: Feynman-Kac Monte Carlo (eqs. 25-30
// with the SDE of eq. 53, Section 2.4 eqs. 36-37) and the inverse-multiquadric
// finalisation (eqs. 19-22); boundary (junction) rows.
//
// Path kernel: one path per lane.  A wavefront owns one (knot, batch) unit and
// refills lanes whose path has exited with the next path index of the batch,
// in lane order, so the schedule (and every sum) is deterministic.  Step k of
// path p from knot i draws Philox4x32-10 at counter (k, p, i, 0) with key
// (seed lo, seed hi); two 53-bit uniforms on (0, 1] feed Box-Muller.  A step
// whose end point stays inside the circle and the domain is accepted; otherwise
// the path exits at the first crossing of the segment with the circle or with
// a boundary piece that the end point violates.  Exits on Gamma_m add
// Y phi_l(theta) to S_l for every arc knot l (H_j = sum_l (K^-1)_lj phi_l is
// applied once per knot in the finalisation); exits on the boundary add g Y;
// every path adds Z.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "mc.h"

namespace pdd {

namespace {

constexpr int kW = 64;
constexpr int kCoefGeneral = 0, kCoefConst = 1, kCoefWave = 2;

// Lane l's double, read by every lane (l wavefront-uniform).
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

struct Philox4 { uint32_t v[4]; };

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1) {
  // Salmon et al. (SC'11): ten rounds of two 32x32 -> 64 multiplies with key
  // schedule k += (0x9E3779B9, 0xBB67AE85).
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Philox4 r;
  r.v[0] = c0; r.v[1] = c1; r.v[2] = c2; r.v[3] = c3;
  return r;
}

// (m + 1) 2^-53 with the 53-bit integer m = hi * 2^21 + lo / 2^11
__device__ __forceinline__ double unit53(uint32_t hi, uint32_t lo) {
  const uint64_t m = ((uint64_t)hi << 21) | (uint64_t)(lo >> 11);
  return ((double)m + 1.0) * 1.1102230246251565404236316680908203125e-16;
}

// positive root t of |p + t d - c| = r for p inside the circle
__device__ __forceinline__ double exit_root(double px, double py, double dx, double dy, double cx,
                                            double cy, double r) {
  const double a = dx * dx + dy * dy;
  const double ex = px - cx, ey = py - cy;
  const double b = ex * dx + ey * dy;
  const double c = ex * ex + ey * ey - r * r;
  const double sq = sqrt(fmax(b * b - a * c, 0.0));
  return (b > 0.0) ? -c / (b + sq) : (sq - b) / a;
}

// smaller positive root of |p + t d - c| = r for p outside the circle
__device__ __forceinline__ double entry_root(double px, double py, double dx, double dy, double cx,
                                             double cy, double r) {
  const double a = dx * dx + dy * dy;
  const double ex = px - cx, ey = py - cy;
  const double b = ex * dx + ey * dy;
  const double c = ex * ex + ey * ey - r * r;
  const double sq = sqrt(fmax(b * b - a * c, 0.0));
  return (b < 0.0) ? c / (sq - b) : (-b - sq) / a;
}

// first crossing of segment p -> q with each domain boundary piece that q violates
__device__ __forceinline__ double domain_exit(const pdd_domain& d, double px, double py, double qx,
                                              double qy) {
  const double dx = qx - px, dy = qy - py;
  double t = INFINITY;
  if (d.kind == PDD_DOMAIN_BOX) {
    if (qx <= d.x0) t = fmin(t, (d.x0 - px) / dx);
    if (qx >= d.x1) t = fmin(t, (d.x1 - px) / dx);
    if (qy <= d.y0) t = fmin(t, (d.y0 - py) / dy);
    if (qy >= d.y1) t = fmin(t, (d.y1 - py) / dy);
  } else {
    const double ex = qx - d.cx, ey = qy - d.cy;
    if (ex * ex + ey * ey >= d.R * d.R) t = fmin(t, exit_root(px, py, dx, dy, d.cx, d.cy, d.R));
    for (int h = 0; h < d.n_holes; ++h) {
      const double hx = d.holes[h][0], hy = d.holes[h][1], hr = d.holes[h][2];
      const double fx = qx - hx, fy = qy - hy;
      if (fx * fx + fy * fy <= hr * hr) t = fmin(t, entry_root(px, py, dx, dy, hx, hy, hr));
    }
  }
  return t;
}

// -zeta(1/2) / sqrt(2 pi): the mean overshoot constant of the shifted scheme
constexpr double kGmC0 = 0.5825971579390106;

// Boundary-shifted Euler (Gobet and Menozzi, SPA 120 (2010)): an end point q
// inside Omega_m closer to a boundary piece (the circle; box sides, or the
// outer circle and holes of a disk) than c0 sqrt(h) |sigma^T n| stops the
// path.  Returns whether it does, the projection of q onto the nearest such
// piece (ties: the circle first, then the pieces in that order) and whether
// that piece is the circle.  sigma is the left point's Cholesky factor.
__device__ __forceinline__ bool shift_stop(const pdd_domain& d, double qx, double qy, double cx, double cy,
                                           double r, double a11, double a21, double a22, double sqh,
                                           double& sx, double& sy, bool& gam) {
  double best = INFINITY;
  auto consider = [&](double dist, double nx, double ny, double px, double py, bool circ) {
    const double t1 = a11 * nx + a21 * ny, t2 = a22 * ny;
    const double band = kGmC0 * sqh * sqrt(t1 * t1 + t2 * t2);
    if (dist < band && dist < best) {
      best = dist;
      sx = px;
      sy = py;
      gam = circ;
    }
  };
  {
    const double ex = qx - cx, ey = qy - cy;
    const double rho = sqrt(ex * ex + ey * ey);
    const double nx = ex / rho, ny = ey / rho;
    consider(r - rho, nx, ny, cx + r * nx, cy + r * ny, true);
  }
  if (d.kind == PDD_DOMAIN_BOX) {
    consider(qx - d.x0, -1.0, 0.0, d.x0, qy, false);
    consider(d.x1 - qx, 1.0, 0.0, d.x1, qy, false);
    consider(qy - d.y0, 0.0, -1.0, qx, d.y0, false);
    consider(d.y1 - qy, 0.0, 1.0, qx, d.y1, false);
  } else {
    {
      const double fx = qx - d.cx, fy = qy - d.cy;
      const double dd = sqrt(fx * fx + fy * fy);
      const double ux = fx / dd, uy = fy / dd;
      consider(d.R - dd, ux, uy, d.cx + d.R * ux, d.cy + d.R * uy, false);
    }
    for (int hh = 0; hh < d.n_holes; ++hh) {
      const double hx = d.holes[hh][0], hy = d.holes[hh][1], hr = d.holes[hh][2];
      const double fx = qx - hx, fy = qy - hy;
      const double dd = sqrt(fx * fx + fy * fy);
      const double ux = fx / dd, uy = fy / dd;
      consider(dd - hr, -ux, -uy, hx + hr * ux, hy + hr * uy, false);
    }
  }
  return best < INFINITY;
}

// Whether q (inside Omega_m, at distance dc from the circle) lies within
// `band` of the circle or of a piece of the domain boundary.
__device__ __forceinline__ bool near_boundary(const pdd_domain& d, double qx, double qy, double dc, double band) {
  if (dc < band) return true;
  if (d.kind == PDD_DOMAIN_BOX)
    return qx - d.x0 < band || d.x1 - qx < band || qy - d.y0 < band || d.y1 - qy < band;
  const double fx = qx - d.cx, fy = qy - d.cy;
  if (d.R - sqrt(fx * fx + fy * fy) < band) return true;
  for (int hh = 0; hh < d.n_holes; ++hh) {
    const double gx = qx - d.holes[hh][0], gy = qy - d.holes[hh][1];
    if (sqrt(gx * gx + gy * gy) - d.holes[hh][2] < band) return true;
  }
  return false;
}

// COEF: kCoefGeneral, kCoefConst (constant coefficients, Laplace-type
// problems) or kCoefWave (every variable field a sine sum with integer wave
// numbers, evaluated from the per-lane power table).
template <int COEF, bool SHIFT>
__device__ __forceinline__ void paths_body(const DevProblem* __restrict__ P, const McArgs& a) {
  const int lane = threadIdx.x & 63;
  const int64_t unit = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (unit >= a.n_units) return;                     // whole wavefront leaves together
  const int B = a.n_batches;
  const int slot = (int)(unit / B), batch = (int)(unit - (int64_t)slot * B);
  const int knot = a.mc_knots[slot];
  const int m = a.assigned[knot];
  const int64_t Ptot = a.paths;
  const int64_t p_lo = (batch * Ptot + B - 1) / B;
  const int64_t p_hi = ((batch + 1) * Ptot + B - 1) / B;
  const double cx = a.cx[m], cy = a.cy[m], r = a.rad[m], r2 = r * r;
  const double h = a.h_circle ? a.h_circle[m] : a.h;
  const double sqh = sqrt(h);
  const double t0 = a.arc0[m], t1 = a.arc1[m];
  const double c2 = a.rbf_c2[m];
  const int64_t alo = a.knot_off[m];
  const int n_arc = (int)(a.knot_off[m + 1] - alo);
  const double x0 = a.kx[knot], y0 = a.ky[knot];
  const uint32_t key0 = (uint32_t)a.seed, key1 = (uint32_t)(a.seed >> 32);
  const int cap = a.step_cap;
  const DevProblem& PP = *P;
  // this lane's table of the powers of e^{2 pi i x}, e^{2 pi i y} (variable
  // coefficients with integer wave numbers)
  constexpr bool CONST_COEF = COEF == kCoefConst;
  __shared__ double2 wtab[COEF == kCoefWave ? 2 * (kWaveMax + 1) : 1][256];
  const WaveTab tab{&wtab[0][threadIdx.x], 256};

  // arc knots in chunks of 64 (lane l holds knot l + 64 s); chunks is uniform
  const int chunks = (n_arc + kW - 1) / kW;
  double th_arc[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int idx = lane + kW * s;
    th_arc[s] = (idx < n_arc) ? a.ktheta[alo + idx] : 0.0;
  }
  double acc_phi[3] = {0.0, 0.0, 0.0};
  double acc_g = 0.0;
  uint64_t steps = 0, capped = 0, gamma_exits = 0;

  // constant coefficients (Laplace-type problems)
  double s11 = 0, s21 = 0, s22 = 0, kbx = 0, kby = 0, kc = 0, kf = 0;
  if (CONST_COEF) {
    s11 = sqrt(PP.k[0]);
    s21 = PP.k[1] / s11;
    s22 = sqrt(PP.k[2] - s21 * s21);
    kbx = PP.k[3]; kby = PP.k[4]; kc = PP.k[5]; kf = PP.k[6];
  }
  const double eck = exp(kc * h);

  int64_t p = p_lo + lane;
  bool active = p < p_hi;
  int64_t next = p_lo + kW;
  uint32_t k = 0;
  double x = x0, y = y0, Y = 1.0, Z = 0.0;

  while (__any(active)) {
    bool exited = false, on_gamma = false;
    double th_e = 0.0, w_e = 0.0;
    if (active) {
      const Philox4 rv = philox4x32_10(k, (uint32_t)p, (uint32_t)knot, 0u, key0, key1);
      const double u1 = unit53(rv.v[0], rv.v[1]);
      const double u2 = unit53(rv.v[2], rv.v[3]);
      const double rad = sqrt(-2.0 * log(u1));
      double sn, cs;
      sincos(kTwoPiD * u2, &sn, &cs);
      const double n1 = rad * cs, n2 = rad * sn;
      double bx, by, cc, ff, a11, a21, a22, ec;
      if (CONST_COEF) {
        bx = kbx; by = kby; cc = kc; ff = kf; a11 = s11; a21 = s21; a22 = s22; ec = eck;
      } else {
        double co[7];
        if (COEF == kCoefWave) coefficients_wave(PP, x, y, co, tab);
        else coefficients_at(PP, x, y, co);
        a11 = sqrt(co[0]);
        a21 = co[1] / a11;
        a22 = sqrt(co[2] - a21 * a21);
        bx = co[3]; by = co[4]; cc = co[5]; ff = co[6];
        ec = exp(cc * h);
      }
      const double qx = x + bx * h + sqh * (a11 * n1);
      const double qy = y + by * h + sqh * (a21 * n1 + a22 * n2);
      const double ex = qx - cx, ey = qy - cy;
      const bool in_c = ex * ex + ey * ey < r2;
      const bool in_d = in_domain(PP.dom, qx, qy);
      bool stop = false, s_gam = false;
      double s_x = 0.0, s_y = 0.0;
      // |sigma^T n| <= |sigma|_F: end points farther than that band from every
      // piece cannot stop, and most steps are decided without the normals
      if (SHIFT && in_c && in_d &&
          near_boundary(PP.dom, qx, qy, r - sqrt(ex * ex + ey * ey),
                        kGmC0 * sqh * sqrt(a11 * a11 + a21 * a21 + a22 * a22) * (1.0 + 1e-12)))
        stop = shift_stop(PP.dom, qx, qy, cx, cy, r, a11, a21, a22, sqh, s_x, s_y, s_gam);
      if (in_c && in_d && !stop) {
        Z = Z + ff * Y * h;
        Y = Y * ec;
        x = qx;
        y = qy;
        ++k;
        if ((int64_t)k >= cap) {           // abandoned: reported as PDD_EPATHCAP
          ++capped;
          steps += k;
          exited = true;
        }
      } else {
        double xe, ye, Ye, Ze;
        if (stop) {                        // shifted boundary: stopped after the full step
          xe = s_x;
          ye = s_y;
          Ye = Y * ec;
          Ze = Z + ff * Y * h;
          on_gamma = s_gam;
        } else {
          const double dx = qx - x, dy = qy - y;
          const double tc = in_c ? INFINITY : exit_root(x, y, dx, dy, cx, cy, r);
          const double td = in_d ? INFINITY : domain_exit(PP.dom, x, y, qx, qy);
          const double ts = fmin(fmax(fmin(tc, td), 0.0), 1.0);
          xe = x + ts * dx;
          ye = y + ts * dy;
          Ye = Y * exp(cc * ts * h);
          Ze = Z + ff * Y * ts * h;
          on_gamma = tc <= td;
        }
        double gv = 0.0;
        if (!on_gamma) {
          const DevField& G = PP.fld[F_G];
          if (COEF == kCoefWave && G.kind == PDD_FIELD_SINSUM && G.wave) {
            wave_fill(tab, xe, ye);          // the step's coefficients are done with the table
            gv = sinsum_tab(G, tab);
          } else {
            gv = boundary_value(PP, xe, ye);
          }
        }
        acc_g += (on_gamma ? 0.0 : gv * Ye) + Ze;
        steps += (uint64_t)k + 1;
        exited = true;
        if (on_gamma) {
          ++gamma_exits;
          double th = atan2(ye - cy, xe - cx) - t0;
          th = t0 + (th - kTwoPiD * floor(th / kTwoPiD));
          if (th > t1) th = (th - t1 <= t0 + kTwoPiD - th) ? t1 : t0;
          th_e = th;
          w_e = Ye;
        }
      }
    }
    // accumulate the Gamma exits of this step in lane order
    uint64_t gmask = __ballot(exited && on_gamma);
    while (gmask) {
      const int e = __ffsll((unsigned long long)gmask) - 1;
      gmask &= gmask - 1;
      // e is wavefront-uniform: the exit's angle and weight as scalars
      const double th = readlane_f64(th_e, e);
      const double wt = readlane_f64(w_e, e);
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        if (s < chunks) {
          const double d = th - th_arc[s];
          acc_phi[s] += wt * rsqrt(d * d + c2);
        }
      }
    }
    // refill exited lanes with the next paths of the batch
    const uint64_t emask = __ballot(exited);
    if (exited) {
      const uint64_t below = emask & ((1ull << lane) - 1ull);
      const int64_t pn = next + __popcll(below);
      p = pn;
      active = pn < p_hi;
      k = 0;
      x = x0; y = y0; Y = 1.0; Z = 0.0;
    }
    next += __popcll(emask);
  }
  // deterministic wavefront reductions
  for (int off = 32; off > 0; off >>= 1) {
    acc_g += __shfl_xor(acc_g, off, kW);
    steps += __shfl_xor(steps, off, kW);
    capped += __shfl_xor(capped, off, kW);
    gamma_exits += __shfl_xor(gamma_exits, off, kW);
  }
  double* out = a.out_phi + unit * a.out_stride;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int idx = lane + kW * s;
    if (idx < n_arc) out[idx] = acc_phi[s];
  }
  if (lane == 0) {
    a.out_g[unit] = acc_g;
    a.out_steps[unit] = steps;
    a.out_capped[unit] = capped;
    a.out_gamma[unit] = gamma_exits;
  }
}

template <int COEF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void paths_kernel(
    const DevProblem* __restrict__ P, McArgs a) {
  paths_body<COEF, false>(P, a);
}

// The shifted scheme's extra live values would otherwise push the kernel
// to one wavefront per SIMD.
template <int COEF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void paths_shifted_kernel(
    const DevProblem* __restrict__ P, McArgs a) {
  paths_body<COEF, true>(P, a);
}

// Packed lower-triangle index (j <= i).
__device__ __forceinline__ int tri(int i, int j) { return (i * (i + 1) >> 1) + j; }

// Cholesky factor of the IMQ Gram matrix K_lk = phi_k(theta_l) (eq. 20) of
// each perimeter circle, factorised in LDS and stored as a packed lower
// triangle in `Lf` (stride n_max (n_max + 1) / 2).
__global__ __launch_bounds__(256) void gram_cholesky_kernel(McArgs a, double* __restrict__ Lf,
                                                            int32_t* __restrict__ status) {
  extern __shared__ double sL[];                       // packed lower triangle
  const int pc = blockIdx.x;
  const int m = a.perim_ids[pc];
  const int64_t alo = a.knot_off[m];
  const int n = (int)(a.knot_off[m + 1] - alo);
  const double c2 = a.rbf_c2[m];
  const int tid = threadIdx.x;
  const int np = n * (n + 1) / 2;
  for (int i = 0; i < n; ++i)
    for (int j = tid; j <= i; j += blockDim.x) {
      const double d = a.ktheta[alo + i] - a.ktheta[alo + j];
      sL[tri(i, j)] = 1.0 / sqrt(d * d + c2);
    }
  __shared__ int s_bad;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double d = sL[tri(k, k)];
    const double piv = sqrt(fmax(d, 1e-300));
    __syncthreads();                                   // every thread has read the diagonal
    if (tid == 0) {
      if (!(d > 0.0)) s_bad = 1;
      sL[tri(k, k)] = piv;
    }
    const double inv = 1.0 / piv;
    for (int i = k + 1 + tid; i < n; i += blockDim.x) sL[tri(i, k)] *= inv;
    __syncthreads();
    // trailing update of the lower triangle, rows and columns > k
    const int rem = n - k - 1;
    const int cnt = rem * (rem + 1) / 2;
    for (int idx = tid; idx < cnt; idx += blockDim.x) {
      // idx -> (ii, jj) with jj <= ii < rem
      int ii = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
      while ((ii + 1) * (ii + 2) / 2 <= idx) ++ii;
      while (ii * (ii + 1) / 2 > idx) --ii;
      const int jj = idx - ii * (ii + 1) / 2;
      const int i = k + 1 + ii, j = k + 1 + jj;
      sL[tri(i, j)] -= sL[tri(i, k)] * sL[tri(j, k)];
    }
    __syncthreads();
  }
  double* L = Lf + (int64_t)pc * a.gram_stride;
  for (int idx = tid; idx < np; idx += blockDim.x) L[idx] = sL[idx];
  if (tid == 0) status[pc] = s_bad;
}

// Per Monte Carlo knot: K^-1 applied to the total and to each batch's phi sums
// (lane b solves right-hand side b against the packed Cholesky factor staged
// in LDS), rows of C = -K^-1 S / Ntilde, batch standard errors, r and its
// standard error, scattered into the CSR arrays.
__global__ __launch_bounds__(64) void mc_finalize_kernel(McArgs a, const double* __restrict__ Lf,
                                                         double* __restrict__ val,
                                                         double* __restrict__ se,
                                                         double* __restrict__ bvec,
                                                         double* __restrict__ se_b) {
  extern __shared__ double smem[];                    // packed L, then [B + 1][n] solutions
  const int slot = blockIdx.x;
  const int lane = threadIdx.x;
  const int knot = a.mc_knots[slot];
  const int m = a.assigned[knot];
  const int pc = a.perim_pos[m];
  const int64_t alo = a.knot_off[m];
  const int n = (int)(a.knot_off[m + 1] - alo);
  const int B = a.n_batches;
  const int np = n * (n + 1) / 2;
  double* sL = smem;
  double* sx = smem + np;
  const double* L = Lf + (int64_t)pc * a.gram_stride;
  for (int idx = lane; idx < np; idx += 64) sL[idx] = L[idx];
  const int64_t Ptot = a.paths;
  const int64_t u0 = (int64_t)slot * B;
  // right-hand sides: lane b < B -> batch mean, lane B -> overall mean
  for (int idx = lane; idx < (B + 1) * n; idx += 64) {
    const int b = idx / n, j = idx - b * n;
    double v;
    if (b < B) {
      const int64_t cnt = ((b + 1) * Ptot + B - 1) / B - (b * Ptot + B - 1) / B;
      v = a.out_phi[(u0 + b) * a.out_stride + j] / (double)cnt;
    } else {
      v = 0.0;
      for (int bb = 0; bb < B; ++bb) v += a.out_phi[(u0 + bb) * a.out_stride + j];
      v /= (double)Ptot;
    }
    sx[idx] = v;
  }
  __syncthreads();
  if (lane <= B) {
    double* x = sx + (int64_t)lane * n;
    for (int i = 0; i < n; ++i) {             // L z = y
      const double* Li = sL + tri(i, 0);
      double v = x[i];
      for (int j = 0; j < i; ++j) v -= Li[j] * x[j];
      x[i] = v / Li[i];
    }
    for (int i = n - 1; i >= 0; --i) {        // L^T x = z
      double v = x[i];
      for (int j = i + 1; j < n; ++j) v -= sL[tri(j, i)] * x[j];
      x[i] = v / sL[tri(i, i)];
    }
  }
  __syncthreads();
  const int64_t rp = a.rowptr[knot];
  const int shift = (knot < alo) ? 1 : 0;
  for (int j = lane; j < n; j += 64) {
    const double tot = -sx[(int64_t)B * n + j];
    double mean = 0.0;
    for (int b = 0; b < B; ++b) mean += -sx[(int64_t)b * n + j];
    mean /= B;
    double var = 0.0;
    for (int b = 0; b < B; ++b) {
      const double d = -sx[(int64_t)b * n + j] - mean;
      var += d * d;
    }
    val[rp + shift + j] = tot;
    se[rp + shift + j] = sqrt(var / (B - 1) / B);
  }
  if (lane == 0) {
    val[rp + (shift ? 0 : n)] = 1.0;
    se[rp + (shift ? 0 : n)] = 0.0;
    double tot = 0.0, mean = 0.0, var = 0.0;
    for (int b = 0; b < B; ++b) tot += a.out_g[u0 + b];
    for (int b = 0; b < B; ++b) {
      const int64_t cnt = ((b + 1) * Ptot + B - 1) / B - (b * Ptot + B - 1) / B;
      mean += a.out_g[u0 + b] / (double)cnt;
    }
    mean /= B;
    for (int b = 0; b < B; ++b) {
      const int64_t cnt = ((b + 1) * Ptot + B - 1) / B - (b * Ptot + B - 1) / B;
      const double d = a.out_g[u0 + b] / (double)cnt - mean;
      var += d * d;
    }
    bvec[knot] = tot / (double)Ptot;
    se_b[knot] = sqrt(var / (B - 1) / B);
  }
}

__global__ void boundary_rows_kernel(const DevProblem* __restrict__ P, const int32_t* __restrict__ ids,
                                     int32_t count, const double* __restrict__ kx,
                                     const double* __restrict__ ky, const int64_t* __restrict__ rowptr,
                                     double* __restrict__ val, double* __restrict__ se,
                                     double* __restrict__ bvec, double* __restrict__ se_b) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int i = ids[t];
  val[rowptr[i]] = 1.0;
  se[rowptr[i]] = 0.0;
  bvec[i] = boundary_value(*P, kx[i], ky[i]);
  se_b[i] = 0.0;
}

}  // namespace

void launch_mc_paths(const DevProblem* P, const DevProblem& host, const McArgs& a, hipStream_t st) {
  if (a.n_units == 0) return;
  const unsigned blocks = (unsigned)((a.n_units + 3) / 4);
  const bool shift = a.scheme == 1;
  typedef void (*Kern)(const DevProblem*, McArgs);
  Kern k;
  if (host.const_coef) k = shift ? paths_shifted_kernel<kCoefConst> : paths_kernel<kCoefConst>;
  else if (host.wave_all) k = shift ? paths_shifted_kernel<kCoefWave> : paths_kernel<kCoefWave>;
  else k = shift ? paths_shifted_kernel<kCoefGeneral> : paths_kernel<kCoefGeneral>;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, st, P, a);
}

void launch_gram_cholesky(const McArgs& a, int32_t n_perim, double* Lf, int32_t* status,
                          hipStream_t st) {
  if (n_perim == 0) return;
  const size_t shm = sizeof(double) * (size_t)a.gram_stride;
  hipFuncSetAttribute((const void*)gram_cholesky_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)shm);
  hipLaunchKernelGGL(gram_cholesky_kernel, dim3(n_perim), dim3(256), shm, st, a, Lf, status);
}

void launch_mc_finalize(const McArgs& a, int32_t n_mc, int32_t max_arc, const double* Lf,
                        double* val, double* se, double* b, double* se_b, hipStream_t st) {
  if (n_mc == 0) return;
  const size_t shm = sizeof(double) * ((size_t)a.gram_stride + (size_t)(a.n_batches + 1) * max_arc);
  hipFuncSetAttribute((const void*)mc_finalize_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)shm);
  hipLaunchKernelGGL(mc_finalize_kernel, dim3(n_mc), dim3(64), shm, st, a, Lf, val, se, b, se_b);
}

void launch_boundary_rows(const DevProblem* P, const int32_t* ids, int32_t count,
                          const double* kx, const double* ky, const int64_t* rowptr, double* val,
                          double* se, double* b, double* se_b, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL(boundary_rows_kernel, dim3((count + 255) / 256), dim3(256), 0, st, P, ids,
                     count, kx, ky, rowptr, val, se, b, se_b);
}

}  // namespace pdd
