// Adjoint of the floating-row assembly with respect to the node samples of
// the coefficients (the derivative of the discrete map; not in the paper).
//
// For floating circle m with assigned knots K_m, interpolation weights E_m
// (rows e_i over the interior nodes) and ring weights:
//   y   = E_m^T lambda_Km
//   mu  = A_II^-T y            (transpose solves on the stored LU of S A_II,
//                               S = row equilibration: mu = S (S A_II)^-T y)
//   w_B = H u_Xi,   w_I = W[:, M] - W[:, :M] u_Xi   (local solution at u)
//   dL/d coef_q = -mu_q (d row_q / d coef_q) . [w_I; w_B],   dL/d f_q = -mu_q
// where row_q is the collocation row of eq. 40 at node q, linear in each of
// the node's coefficient samples.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "runtime.h"

namespace pdd {

namespace {

constexpr int kAdjThreads = 256;
constexpr int kAdjKnots = 32;
constexpr int kTri = 32;

struct AdjArgs {
  BucketTables T;
  ChunkDesc C;
  const double* A;           // factors + W, [count][n][ld]
  int64_t stride;
  const int32_t* piv;        // [count][n]
  const double* rowscale;    // [count][n]
  const double* u;
  const double* lambda;
  double* g[7];              // axx, axy, ayy, bx, by, c, f (node layout), may be null
};

// Lane l's value of a double, l wavefront-uniform.
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Dynamic LDS layout (doubles): y[n] | wI[n] | wB[Nt] | uX[M] | one region shared by the phases:
//   knots: lx[32][Nc+1] | lt[32][Nt] | per-knot rho, phi, lambda, weight sum (4 x 32) | exact index
//   interchanges: piv (n ints);  gradients: G[(Nc+1) Nt]
// (about 39 KB at n = 1024: four workgroups per CU)
__global__ __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(4))) void adjoint_kernel(AdjArgs a) {
  extern __shared__ double sh[];
  const BucketTables& T = a.T;
  const int n = T.n, Nt = T.Nt, Nr = T.Nr, Nc = T.Nc, Nc1 = T.Nc + 1, M = T.M, ld = T.ld;
  const int half = Nt / 2;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int ci = blockIdx.x;
  const int f = a.C.fl[ci];
  const int m = a.C.float_ids[f];
  const double* A = a.A + (int64_t)ci * a.stride;
  const int32_t* piv = a.piv + (int64_t)ci * n;
  const double* sc = a.rowscale + (int64_t)ci * n;
  double* y = sh;
  double* wI = y + n;
  double* wB = wI + n;
  double* uX = wB + Nt;
  double* reg = uX + M;
  double* G = reg;
  double* lx = reg;
  double* lt = lx + kAdjKnots * Nc1;
  double* kr = lt + kAdjKnots * Nt;           // per-knot rho, phi, lambda, weight sum, exact
  double* kp = kr + kAdjKnots;
  double* kw = kp + kAdjKnots;
  double* kq = kw + kAdjKnots;
  int* ke = reinterpret_cast<int*>(kq + kAdjKnots);
  int* spiv = reinterpret_cast<int*>(reg);

  // ---- y = E^T lambda over the assigned knots
  for (int q = tid; q < n; q += kAdjThreads) y[q] = 0.0;
  const int64_t klo = a.C.fk_off[f], khi = a.C.fk_off[f + 1];
  const double cxm = a.C.cx[m], cym = a.C.cy[m], rm = a.C.rad[m];
  for (int64_t base = klo; base < khi; base += kAdjKnots) {
    const int cnt = (int)min<int64_t>(kAdjKnots, khi - base);
    __syncthreads();
    if (tid < cnt) {
      const int i = a.C.fk_ids[base + tid];
      const double dx = a.C.kx[i] - cxm, dy = a.C.ky[i] - cym;
      const double rho = sqrt(dx * dx + dy * dy) / rm;
      int exact = -1;
      double ssum = 0.0;
      for (int j = 0; j < Nc1; ++j) {
        const double d = rho - T.xr[j];
        if (d == 0.0) exact = j;
        else ssum += T.bw[j] / d;
      }
      kr[tid] = rho;
      kp[tid] = atan2(dy, dx);
      kw[tid] = a.lambda[i];
      ke[tid] = exact;
      kq[tid] = ssum;
    }
    __syncthreads();
    // lambda is folded into the radial weights; one (knot, node) entry per thread
    for (int idx = tid; idx < cnt * Nc1; idx += kAdjThreads) {
      const int t = idx / Nc1, j = idx - t * Nc1;
      const int exact = ke[t];
      lx[idx] = kw[t] * ((exact >= 0) ? (j == exact ? 1.0 : 0.0)
                                      : (T.bw[j] / (kr[t] - T.xr[j])) / kq[t]);
    }
    const double hstep = kTwoPiD / Nt;
    for (int idx = tid; idx < cnt * Nt; idx += kAdjThreads) {
      const int t = idx / Nt, l = idx - t * Nt;
      // angle difference reduced to [-pi, pi] (the cardinal is 2 pi-periodic)
      double d = kp[t] - hstep * l;
      d -= kTwoPiD * rint(d / kTwoPiD);
      const double x = 0.5 * d;
      double sx, cx;
      sincos(x, &sx, &cx);
      lt[idx] = (fabs(sx) < 1e-15) ? 1.0 : sin(Nt * x) * cx / (Nt * sx);
    }
    __syncthreads();
    for (int q = tid; q < n; q += kAdjThreads) {
      const int k = q / Nt + 1, lp = q - (k - 1) * Nt;
      int lq = lp + half;
      if (lq >= Nt) lq -= Nt;
      double acc = 0.0;
      for (int t = 0; t < cnt; ++t)
        acc += lx[t * Nc1 + k] * lt[t * Nt + lp] + lx[t * Nc1 + (Nc - k)] * lt[t * Nt + lq];
      y[q] += acc;
    }
  }
  __syncthreads();

  // ---- U^T z = y (forward, 32-row blocks: wavefront 0 solves the diagonal
  //      block from its rows held in registers (lane l holds column l), then
  //      every thread removes the block's contribution from its later
  //      entries, all 32 loads of an entry issued at once)
  for (int j0 = 0; j0 < n; j0 += kTri) {
    const int bw = min(kTri, n - j0), j1 = j0 + bw;
    if (w == 0) {
      double row[kTri];
#pragma unroll
      for (int j = 0; j < kTri; ++j) {
        const bool ok = j < bw && lane < bw;
        const double v = A[ok ? (int64_t)(j0 + j) * ld + j0 + lane : 0];
        row[j] = ok ? v : 0.0;
      }
      double yi = (lane < bw) ? y[j0 + lane] : 0.0;
#pragma unroll
      for (int j = 0; j < kTri; ++j) {
        if (j < bw) {
          const double zj = readlane_f64(yi, j) / readlane_f64(row[j], j);
          if (lane == j) yi = zj;
          else if (lane > j) yi -= row[j] * zj;
        }
      }
      if (lane < bw) y[j0 + lane] = yi;
    }
    __syncthreads();
    for (int i = j1 + tid; i < n; i += kAdjThreads) {
      double acc = 0.0;
#pragma unroll
      for (int h = 0; h < kTri; h += kTri / 2) {
        double v[kTri / 2];
#pragma unroll
        for (int j = 0; j < kTri / 2; ++j) {
          const double x = A[h + j < bw ? (int64_t)(j0 + h + j) * ld + i : 0];
          v[j] = h + j < bw ? x : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kTri / 2; ++j)
          if (h + j < bw) acc += v[j] * y[j0 + h + j];
      }
      y[i] -= acc;
    }
    __syncthreads();
  }
  // ---- L^T x = z (backward, unit diagonal, same blocking)
  for (int j1 = n; j1 > 0; j1 -= kTri) {
    const int j0 = max(0, j1 - kTri), bw = j1 - j0;
    if (w == 0) {
      double row[kTri];
#pragma unroll
      for (int j = 0; j < kTri; ++j) {
        const bool ok = j < bw && lane < bw;
        const double v = A[ok ? (int64_t)(j0 + j) * ld + j0 + lane : 0];
        row[j] = ok ? v : 0.0;
      }
      double yi = (lane < bw) ? y[j0 + lane] : 0.0;
#pragma unroll
      for (int j = kTri - 1; j >= 0; --j) {
        if (j < bw) {
          const double xj = readlane_f64(yi, j);
          if (lane < j) yi -= row[j] * xj;
        }
      }
      if (lane < bw) y[j0 + lane] = yi;
    }
    __syncthreads();
    for (int i = tid; i < j0; i += kAdjThreads) {
      double acc = 0.0;
#pragma unroll
      for (int h = 0; h < kTri; h += kTri / 2) {
        double v[kTri / 2];
#pragma unroll
        for (int j = 0; j < kTri / 2; ++j) {
          const double x = A[h + j < bw ? (int64_t)(j0 + h + j) * ld + i : 0];
          v[j] = h + j < bw ? x : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kTri / 2; ++j)
          if (h + j < bw) acc += v[j] * y[j0 + h + j];
      }
      y[i] -= acc;
    }
    __syncthreads();
  }
  // ---- undo the row interchanges (P^T: the swaps kk <-> piv[kk] for kk
  //      descending): every thread follows its own entries through the swap
  //      sequence and writes each to its final slot; then mu = S nu
  for (int q = tid; q < n; q += kAdjThreads) spiv[q] = piv[q];
  __syncthreads();
  for (int b0 = 0; b0 < n; b0 += 8 * kAdjThreads) {
    int pos[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) pos[e] = b0 + tid + kAdjThreads * e;
#pragma unroll 4
    for (int kk = n - 1; kk >= 0; --kk) {
      const int p = spiv[kk];
#pragma unroll
      for (int e = 0; e < 8; ++e) pos[e] = (pos[e] == kk) ? p : (pos[e] == p ? kk : pos[e]);
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int i = b0 + tid + kAdjThreads * e;
      if (i < n) wI[pos[e]] = y[i];
    }
  }
  __syncthreads();
  for (int q = tid; q < n; q += kAdjThreads) y[q] = wI[q] * sc[q];
  __syncthreads();

  // ---- local solution at u: w_B = H u_Xi, w_I = W[:, M] - W[:, :M] u_Xi
  const int64_t slo = a.C.knot_off[m];
  for (int j = tid; j < M; j += kAdjThreads) uX[j] = a.u[slo + j];
  __syncthreads();
  for (int l = tid; l < Nt; l += kAdjThreads) {
    double acc = 0.0;
    for (int j = 0; j < M; ++j) acc += T.H[(int64_t)l * M + j] * uX[j];
    wB[l] = acc;
  }
  for (int q = tid; q < n; q += kAdjThreads) {
    const double* Wq = A + (int64_t)q * ld + n;
    double acc = Wq[M];
    for (int j = 0; j < M; ++j) acc -= Wq[j] * uX[j];
    wI[q] = acc;
  }
  __syncthreads();
  // full-grid value at radial index j, angular index l
  auto wf = [&](int j, int l) -> double {
    if (j == 0) return wB[l];
    if (j <= Nr) return wI[(j - 1) * Nt + l];
    int lq = l + half;
    if (lq >= Nt) lq -= Nt;
    if (j < Nc) return wI[(Nc - j - 1) * Nt + lq];
    return wB[lq];
  };
  // G(j, l) = sum_l' d1t[l - l'] w(j, l')   (angular derivative on every radial line)
  for (int idx = tid; idx < Nc1 * Nt; idx += kAdjThreads) {
    const int j = idx / Nt, l = idx - j * Nt;
    double acc = 0.0;
    for (int lp = 0; lp < Nt; ++lp) {
      int dl = l - lp;
      if (dl < 0) dl += Nt;
      acc += T.d1t[dl] * wf(j, lp);
    }
    G[idx] = acc;
  }
  __syncthreads();

  // ---- per-node gradients
  const int64_t node0 = a.C.node_off[f];
  const double r = rm, r2 = r * r;
  for (int q = tid; q < n; q += kAdjThreads) {
    const int jr = q / Nt + 1, l = q - (jr - 1) * Nt;
    const double* Drow = T.Dr + (int64_t)(jr - 1) * Nc1;
    const double* D2row = T.D2r + (int64_t)(jr - 1) * Nc1;
    double w_rr = 0.0, w_r = 0.0, w_rt = 0.0, w_tt = 0.0;
    for (int j = 0; j < Nc1; ++j) {
      const double v = wf(j, l);
      w_rr += D2row[j] * v;
      w_r += Drow[j] * v;
      w_rt += Drow[j] * G[j * Nt + l];
    }
    for (int lp = 0; lp < Nt; ++lp) {
      int dl = l - lp;
      if (dl < 0) dl += Nt;
      w_tt += T.d2t[dl] * wf(jr, lp);
    }
    const double w_t = G[jr * Nt + l];
    const double rho = T.xr[jr];
    const double C = T.cs[l], S = T.sn[l];
    const double CC = C * C, SS = S * S, SC = S * C, D2 = CC - SS;
    const double ir2 = 1.0 / r2, irr = 1.0 / (rho * r2), irr2 = 1.0 / (rho * rho * r2);
    const double mu = y[q];
    const double g_axx = 0.5 * CC * ir2 * w_rr + 0.5 * SS * irr * w_r + 0.5 * SS * irr2 * w_tt -
                         SC * irr * w_rt + SC * irr2 * w_t;
    const double g_axy = SC * ir2 * w_rr - SC * irr * w_r - SC * irr2 * w_tt + D2 * irr * w_rt -
                         D2 * irr2 * w_t;
    const double g_ayy = 0.5 * SS * ir2 * w_rr + 0.5 * CC * irr * w_r + 0.5 * CC * irr2 * w_tt +
                         SC * irr * w_rt - SC * irr2 * w_t;
    const double g_bx = C / r * w_r - S / (rho * r) * w_t;
    const double g_by = S / r * w_r + C / (rho * r) * w_t;
    const double vals[7] = {g_axx, g_axy, g_ayy, g_bx, g_by, wI[q], 1.0};
#pragma unroll
    for (int k = 0; k < 7; ++k)
      if (a.g[k]) a.g[k][node0 + q] = -mu * vals[k];
  }
  (void)w;
}

}  // namespace

// Rule AVERAGED: the multiplier of each pair row is that of its knot's row.
__global__ void gather_pairs_kernel(int64_t np, const int32_t* __restrict__ pair_knot,
                                    const double* __restrict__ x, double* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < np) out[q] = x[pair_knot[q]];
}

pdd_status backward_impl(pdd_system sys, const double* u, const double* lambda, double* const g[7],
                         double* g_r, hipStream_t st) {
  const bool avg = sys->cover->H.pairs != nullptr;
  // r enters C u = r linearly: dL/dr = lambda for every row
  if (g_r && sys->cover->H.N() > 0)
    PDD_HIP(hipMemcpyAsync(g_r, lambda, sizeof(double) * (size_t)sys->cover->H.N(), hipMemcpyDefault, st));
  const DeviceCover& D = avg ? sys->cover->DP : sys->cover->D;
  if (sys->factors.empty() && !sys->recompute && !sys->cover->H.float_ids.empty())
    return fail(PDD_EINVAL, "pdd_assemble_G_backward: assemble with keep_factors to differentiate");
  // Row i of C is the sum of its pair rows, so the gradient is that of the
  // pair rows with every pair taking its knot's multiplier.
  DevBuf pair_lambda;
  struct SyncOnExit {
    hipStream_t s;
    bool on;
    ~SyncOnExit() { if (on) (void)hipStreamSynchronize(s); }   // before pair_lambda is freed
  } sync_guard{st, avg};
  if (avg) {
    const int64_t np = sys->cover->H.pairs->N();
    pair_lambda.alloc(std::max<int64_t>(1, np) * sizeof(double));
    if (np > 0)
      hipLaunchKernelGGL(gather_pairs_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, np,
                         D.pair_knot.ptr<int32_t>(), lambda, pair_lambda.ptr<double>());
    PDD_HIP(hipGetLastError());
    lambda = pair_lambda.ptr<double>();
  }
  auto run = [&](const BucketFactors& F) -> pdd_status {
    const BucketData& bk = *D.buckets[F.bucket];
    AdjArgs a{};
    a.T = bk.T;
    a.C = D.chunk(bk, F.first, F.count);
    a.A = F.A.ptr<double>();
    a.stride = F.stride;
    a.piv = F.piv.ptr<int32_t>();
    a.rowscale = F.rowscale.ptr<double>();
    a.u = u;
    a.lambda = lambda;
    for (int k = 0; k < 7; ++k) a.g[k] = g[k];
    const size_t region = std::max({(size_t)kAdjKnots * (bk.Nc + 1 + bk.Nt) + 4 * kAdjKnots + kAdjKnots / 2,
                                    (size_t)(bk.Nc + 1) * bk.Nt, ((size_t)bk.n + 1) / 2});
    const size_t shm = sizeof(double) * ((size_t)2 * bk.n + bk.Nt + bk.M + region);
    if (shm > 160 * 1024) return fail(PDD_EINVAL, "pdd_assemble_G_backward: bucket too large");
    (void)hipFuncSetAttribute((const void*)adjoint_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL(adjoint_kernel, dim3(F.count), dim3(kAdjThreads), shm, st, a);
    PDD_HIP(hipGetLastError());
    return PDD_OK;
  };
  if (!sys->recompute) {
    for (const auto& fp : sys->factors) {
      const pdd_status ps = run(*fp);
      if (ps != PDD_OK) return ps;
    }
    return PDD_OK;
  }
  // The factors did not fit the budget at assembly: rebuild them chunk by
  // chunk from the system's own copy of the node samples (the same kernels,
  // so the same factors) and differentiate each chunk before the next.
  const int64_t sum_n = sys->cover->H.sum_n;
  NodeSamples S{};
  for (int t = 0; t < 7; ++t) S.s[t] = sys->samples.ptr<double>() + (int64_t)t * sum_n;
  LuScratch ws;
  for (size_t bi = 0; bi < D.buckets.size(); ++bi) {
    const BucketData& bk = *D.buckets[bi];
    const int32_t chunk = (int32_t)std::min<int64_t>(
        bk.count, std::max<int64_t>(1, sys->budget / factor_bytes_per_circle(bk)));
    BucketFactors f;
    f.bucket = (int32_t)bi;
    alloc_factors(f, bk, chunk);
    for (int32_t first = 0; first < bk.count; first += chunk) {
      const int32_t cnt = std::min(chunk, bk.count - first);
      factor_chunk(D, bk, S, sys->plan, f, first, cnt, ws, st, nullptr, nullptr, nullptr);
      const pdd_status ps = run(f);
      if (ps != PDD_OK) return ps;
    }
    PDD_HIP(hipStreamSynchronize(st));   // before the chunk buffers are freed
  }
  return PDD_OK;
}

}  // namespace pdd

using namespace pdd;

extern "C" pdd_status pdd_assemble_G_backward(pdd_system sys, const double* u, const double* lambda,
                                              double* g_axx, double* g_axy, double* g_ayy,
                                              double* g_bx, double* g_by, double* g_c, double* g_f,
                                              double* g_r, void* stream) {
  if (!sys || !u || !lambda) return fail(PDD_EINVAL, "pdd_assemble_G_backward: null argument");
  try {
    double* const g[7] = {g_axx, g_axy, g_ayy, g_bx, g_by, g_c, g_f};
    return backward_impl(sys, u, lambda, g, g_r, (hipStream_t)stream);
  } catch (const HipError& e) {
    return fail(PDD_EDEVICE, e.what());
  } catch (const std::bad_alloc&) {
    return fail(PDD_ENOMEM, "pdd_assemble_G_backward: out of host memory");
  } catch (const std::exception& e) {
    return fail(PDD_EDEVICE, std::string("pdd_assemble_G_backward: ") + e.what());
  }
}
