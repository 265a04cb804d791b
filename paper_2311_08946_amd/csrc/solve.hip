// Solve of the interfacial system C u = r (and C^T lambda = g for the
// adjoint) by BiCGStab on the device (Remark 2 asks for a distributed Krylov
// solver; the paper's runs use preconditioned GMRES).
//
// The CSR matrix-vector product uses one wavefront per row with a fixed
// reduction order; dot products reduce block partials in a fixed order, so
// repeated solves give bitwise-identical iterates.  The scalars (rho, alpha,
// omega, ...) stay on the device; the host reads one residual per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "runtime.h"

namespace pdd {

namespace {

constexpr int kDotBlocks = 512;
constexpr int kThreads = 256;

// scalar slots in device memory
enum { S_RHO = 0, S_RHO_OLD, S_ALPHA, S_OMEGA, S_RV, S_TS, S_TT, S_RR, S_BB, S_BETA, S_COUNT };

__global__ __launch_bounds__(256) void spmv_kernel(const int64_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ cols,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ y, int64_t N,
                                                   const double* __restrict__ b_minus) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= N) return;
  const int64_t lo = rowptr[row], hi = rowptr[row + 1];
  double acc = 0.0;
  for (int64_t k = lo + lane; k < hi; k += 64) acc += val[k] * x[cols[k]];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) y[row] = b_minus ? b_minus[row] - acc : acc;
}

__global__ void gather_kernel(const int64_t* __restrict__ perm, const double* __restrict__ src,
                              double* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

// partial[b] = sum over this block's strided range of a*b (fixed order)
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double s[kThreads];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  return s[0];
}

__global__ __launch_bounds__(256) void dot2_partial_kernel(const double* __restrict__ a,
                                                           const double* __restrict__ b,
                                                           const double* __restrict__ c,
                                                           const double* __restrict__ d, int64_t n,
                                                           double* __restrict__ part) {
  double v1 = 0.0, v2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    v1 += a[i] * b[i];
    if (c) v2 += c[i] * d[i];
  }
  const double s1 = block_sum(v1);
  __syncthreads();
  const double s2 = block_sum(v2);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1;
    part[kDotBlocks + blockIdx.x] = s2;
  }
}

// Reduces the partials into slot `slot1` (and `slot2`) and updates the
// derived BiCGStab scalars according to `stage`.
__global__ __launch_bounds__(256) void dot_finalize_kernel(const double* __restrict__ part, int nb,
                                                           double* __restrict__ sc, int slot1,
                                                           int slot2, int stage) {
  double v1 = 0.0, v2 = 0.0;
  for (int i = threadIdx.x; i < nb; i += kThreads) {
    v1 += part[i];
    v2 += part[kDotBlocks + i];
  }
  const double s1 = block_sum(v1);
  __syncthreads();
  const double s2 = block_sum(v2);
  if (threadIdx.x == 0) {
    sc[slot1] = s1;
    if (slot2 >= 0) sc[slot2] = s2;
    if (stage == 1) {            // rho known: beta = (rho / rho_old) (alpha / omega)
      const double beta = (sc[S_RHO] / sc[S_RHO_OLD]) * (sc[S_ALPHA] / sc[S_OMEGA]);
      sc[S_BETA] = beta;
      sc[S_RHO_OLD] = sc[S_RHO];
    } else if (stage == 2) {     // (r0, v) known: alpha = rho / (r0, v)
      sc[S_ALPHA] = sc[S_RHO] / sc[S_RV];
    } else if (stage == 3) {     // (t, s), (t, t) known: omega = (t, s) / (t, t)
      sc[S_OMEGA] = (sc[S_TT] > 0.0) ? sc[S_TS] / sc[S_TT] : 0.0;
    }
  }
}

__global__ void update_p_kernel(double* __restrict__ p, const double* __restrict__ r,
                                const double* __restrict__ v, const double* __restrict__ sc,
                                int64_t n, int first) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (first) p[i] = r[i];
  else p[i] = r[i] + sc[S_BETA] * (p[i] - sc[S_OMEGA] * v[i]);
}

__global__ void update_s_kernel(double* __restrict__ s, const double* __restrict__ r,
                                const double* __restrict__ v, const double* __restrict__ sc,
                                int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) s[i] = r[i] - sc[S_ALPHA] * v[i];
}

__global__ void update_xr_kernel(double* __restrict__ x, double* __restrict__ r,
                                 const double* __restrict__ p, const double* __restrict__ s,
                                 const double* __restrict__ t, const double* __restrict__ sc,
                                 int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = sc[S_ALPHA], w = sc[S_OMEGA];
  x[i] = x[i] + a * p[i] + w * s[i];
  r[i] = s[i] - w * t[i];
}

__global__ void copy_kernel(double* __restrict__ d, const double* __restrict__ s, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

__global__ void init_scalars_kernel(double* sc) {
  if (threadIdx.x == 0) {
    for (int k = 0; k < S_COUNT; ++k) sc[k] = 0.0;
    sc[S_RHO_OLD] = 1.0;
    sc[S_ALPHA] = 1.0;
    sc[S_OMEGA] = 1.0;
  }
}

}  // namespace

// Transpose pattern of C: rows of C^T with, for each entry, its position in C.
void ensure_transpose(pdd_cover cover) {
  DeviceCover& D = cover->D;
  if (D.have_transpose) return;
  const HostCover& H = cover->H;
  const int64_t N = H.N(), nnz = H.rowptr.back();
  std::vector<int64_t> rp(N + 1, 0);
  for (int64_t k = 0; k < nnz; ++k) ++rp[H.cols[k] + 1];
  for (int64_t i = 0; i < N; ++i) rp[i + 1] += rp[i];
  std::vector<int32_t> cl(nnz);
  std::vector<int64_t> perm(nnz);
  std::vector<int64_t> fill(rp.begin(), rp.end() - 1);
  for (int64_t i = 0; i < N; ++i)
    for (int64_t k = H.rowptr[i]; k < H.rowptr[i + 1]; ++k) {
      const int64_t pos = fill[H.cols[k]]++;
      cl[pos] = (int32_t)i;
      perm[pos] = k;
    }
  D.rt_rowptr.upload(rp);
  D.rt_cols.upload(cl);
  D.rt_perm.upload(perm);
  D.have_transpose = true;
}

pdd_status solve_impl(pdd_system sys, const double* rhs, double* u, int32_t transpose,
                      const pdd_solve_opts* opts, hipStream_t st, pdd_solve_info* info) {
  const HostCover& H = sys->cover->H;
  DeviceCover& D = sys->cover->D;
  const int64_t N = H.N(), nnz = H.rowptr.back();
  const double rtol = (opts && opts->rtol > 0.0) ? opts->rtol : 1e-12;
  const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 2000;
  const bool guess = opts && opts->use_guess;
  const int64_t* rowptr = D.rowptr.ptr<int64_t>();
  const int32_t* cols = D.cols.ptr<int32_t>();
  const double* val = sys->val.ptr<double>();
  DevBuf valT;
  if (transpose) {
    ensure_transpose(sys->cover);
    valT.alloc(nnz * sizeof(double));
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st,
                       D.rt_perm.ptr<int64_t>(), val, valT.ptr<double>(), nnz);
    rowptr = D.rt_rowptr.ptr<int64_t>();
    cols = D.rt_cols.ptr<int32_t>();
    val = valT.ptr<double>();
  }
  const double* b = rhs ? rhs : sys->b.ptr<double>();
  DevBuf work;
  work.alloc(sizeof(double) * (6 * N + 2 * kDotBlocks + S_COUNT));
  double* r = work.ptr<double>();
  double* r0 = r + N;
  double* p = r0 + N;
  double* v = p + N;
  double* s = v + N;
  double* t = s + N;
  double* part = t + N;
  double* sc = part + 2 * kDotBlocks;
  const unsigned vb = (unsigned)((N + 255) / 256);
  const unsigned rb = (unsigned)((N + 3) / 4);
  const unsigned db = (unsigned)std::min<int64_t>(kDotBlocks, (N + kThreads - 1) / kThreads);
  auto dot = [&](const double* a1, const double* b1, const double* a2, const double* b2, int s1,
                 int s2, int stage) {
    hipLaunchKernelGGL(dot2_partial_kernel, dim3(db), dim3(kThreads), 0, st, a1, b1, a2, b2, N, part);
    hipLaunchKernelGGL(dot_finalize_kernel, dim3(1), dim3(kThreads), 0, st, part, (int)db, sc, s1,
                       s2, stage);
  };
  hipLaunchKernelGGL(init_scalars_kernel, dim3(1), dim3(64), 0, st, sc);
  if (!guess) PDD_HIP(hipMemsetAsync(u, 0, N * sizeof(double), st));
  hipLaunchKernelGGL(spmv_kernel, dim3(rb), dim3(256), 0, st, rowptr, cols, val, u, r, N, b);
  hipLaunchKernelGGL(copy_kernel, dim3(vb), dim3(256), 0, st, r0, r, N);
  dot(b, b, r, r, S_BB, S_RR, 0);
  double host[S_COUNT];
  PDD_HIP(hipMemcpyAsync(host, sc, sizeof(host), hipMemcpyDeviceToHost, st));
  PDD_HIP(hipStreamSynchronize(st));
  const double bnorm = std::sqrt(host[S_BB]);
  double rel = bnorm > 0.0 ? std::sqrt(host[S_RR]) / bnorm : 0.0;
  int it = 0;
  bool ok = bnorm == 0.0 || rel <= rtol;
  if (bnorm == 0.0) PDD_HIP(hipMemsetAsync(u, 0, N * sizeof(double), st));
  // p = v = 0 and rho_old = alpha = omega = 1 make the first update p = r
  PDD_HIP(hipMemsetAsync(p, 0, 2 * N * sizeof(double), st));
  while (!ok && it < max_iter) {
    dot(r0, r, nullptr, nullptr, S_RHO, -1, 1);
    hipLaunchKernelGGL(update_p_kernel, dim3(vb), dim3(256), 0, st, p, r, v, sc, N, 0);
    hipLaunchKernelGGL(spmv_kernel, dim3(rb), dim3(256), 0, st, rowptr, cols, val, p, v, N,
                       (const double*)nullptr);
    dot(r0, v, nullptr, nullptr, S_RV, -1, 2);
    hipLaunchKernelGGL(update_s_kernel, dim3(vb), dim3(256), 0, st, s, r, v, sc, N);
    hipLaunchKernelGGL(spmv_kernel, dim3(rb), dim3(256), 0, st, rowptr, cols, val, s, t, N,
                       (const double*)nullptr);
    dot(t, s, t, t, S_TS, S_TT, 3);
    hipLaunchKernelGGL(update_xr_kernel, dim3(vb), dim3(256), 0, st, u, r, p, s, t, sc, N);
    dot(r, r, nullptr, nullptr, S_RR, -1, 0);
    PDD_HIP(hipGetLastError());
    PDD_HIP(hipMemcpyAsync(host, sc, sizeof(host), hipMemcpyDeviceToHost, st));
    PDD_HIP(hipStreamSynchronize(st));
    ++it;
    rel = std::sqrt(host[S_RR]) / bnorm;
    if (!std::isfinite(rel) || host[S_RV] == 0.0 || host[S_RHO] == 0.0) break;
    ok = rel <= rtol;
  }
  if (info) {
    info->iterations = it;
    info->converged = ok ? 1 : 0;
    info->rel_residual = rel;
  }
  if (!ok)
    return fail(PDD_ENOCONV, "pdd_solve_G: BiCGStab stopped at relative residual " +
                                 std::to_string(rel) + " after " + std::to_string(it) + " iterations");
  return PDD_OK;
}

}  // namespace pdd

using namespace pdd;

extern "C" pdd_status pdd_solve_G(pdd_system sys, const double* rhs, double* u, int32_t transpose,
                                  const pdd_solve_opts* opts, void* stream, pdd_solve_info* info) {
  if (!sys || !u) return fail(PDD_EINVAL, "pdd_solve_G: null argument");
  try {
    return solve_impl(sys, rhs, u, transpose, opts, (hipStream_t)stream, info);
  } catch (const HipError& e) {
    return fail(e.code == hipErrorOutOfMemory ? PDD_ENOMEM : PDD_EDEVICE, e.what());
  } catch (const std::bad_alloc&) {
    return fail(PDD_ENOMEM, "pdd_solve_G: out of host memory");
  }
}
