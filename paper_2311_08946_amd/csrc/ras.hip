// One-level restricted additive Schwarz preconditioner (Section 4, eqs. 42-44)
// and restarted right-preconditioned GMRES (eq. 45) for C u = r.
//
// Set-up: the circles are split geometrically into px x py parts (sorted by
// centre x into slabs of near-equal counts, each slab by centre y), a knot
// belongs to the part of the circle it lies on, and omega_p adds one layer of
// neighbours in the symmetric graph of C.  Every C_p = R_p C R_p^T is gathered
// densely into [C_p | I] (order padded to a multiple of 32 with identity rows)
// and the whole set is factorised by the batched MFMA LU, whose forward
// elimination and back substitution of the identity columns leave C_p^-1 in
// place.  Applying M^-1 is then a batched dense GEMV per part (HBM-bound, the
// inverses read once) and a fixed-order weighted sum per knot (D_p of eq. 43).
//
// GMRES(m): Arnoldi by classical Gram-Schmidt applied twice (two passes of
// one multi-dot and one update each, instead of j + 1 sequential dot/axpy
// pairs); the Givens rotations and the convergence test run on the device in
// one single-thread kernel per iteration, and the host reads the state once
// per batch of iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "runtime.h"

struct pdd_ras_s {
  pdd_system sys = nullptr;
  int32_t P = 0, max_npad = 0;
  bool f32 = false;                     // inverses kept in FP32 (inv32), else in mat
  int64_t total = 0;                    // sum of #omega_p
  std::vector<int64_t> off;             // [P+1] offsets into knots
  std::vector<int32_t> knots;           // omega_p, sorted, concatenated
  std::vector<int32_t> npad;            // padded order of each C_p
  std::vector<int64_t> aoff;            // offset (doubles) of each [C_p | C_p^-1]
  std::vector<int64_t> poff;            // offset of each part's padded vector slots
  std::vector<int64_t> ioff;            // offset (floats) of each part's FP32 inverse
  pdd::DevBuf d_off, d_knots, d_npad, d_aoff, d_poff, d_moff, d_mslot, mat, piv, status, work, t, xg;
  pdd::DevBuf d_ioff, inv32;
};

namespace pdd {

namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kDotBlocks = 512;          // partial sums per multi-dot

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ int64_t find_sorted(const int32_t* __restrict__ a, int64_t n, int32_t key) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return (lo < n && a[lo] == key) ? lo : -1;
}

// [C_p | I] for every part; one wavefront per local row, the matrix zeroed
// beforehand.  Padding rows get a unit diagonal.
__global__ void __launch_bounds__(kBlock) gather_blocks_kernel(
    const int64_t* __restrict__ off, const int32_t* __restrict__ knots, const int32_t* __restrict__ npad,
    const int64_t* __restrict__ aoff, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ cols,
    const double* __restrict__ val, double* __restrict__ mat) {
  const int p = blockIdx.y;
  const int r = blockIdx.x * (kBlock / kWave) + (threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int np = npad[p];
  if (r >= np) return;
  const int64_t o = off[p];
  const int64_t n = off[p + 1] - o;
  const int ld = 2 * np;
  double* A = mat + aoff[p] + (int64_t)r * ld;
  if (r < n) {
    const int32_t i = knots[o + r];
    for (int64_t e = rowptr[i] + lane; e < rowptr[i + 1]; e += kWave) {
      const int64_t c = find_sorted(knots + o, n, cols[e]);
      if (c >= 0) A[c] = val[e];
    }
  } else if (lane == 0) {
    A[r] = 1.0;
  }
  if (lane == 0) A[np + r] = 1.0;
}

// xg_p = x|omega_p, zero-padded to the part's padded order (the rows of the
// stored inverses are zero beyond #omega_p, so the GEMV runs over npad).
__global__ void gather_x_kernel(const int64_t* __restrict__ off, const int32_t* __restrict__ knots,
                                const int32_t* __restrict__ npad, const int64_t* __restrict__ poff,
                                const double* __restrict__ x, double* __restrict__ xg,
                                const int* __restrict__ stop) {
  if (stop && *stop) return;
  const int p = blockIdx.y;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int np = npad[p];
  if (c >= np) return;
  const int64_t o = off[p];
  const int n = (int)(off[p + 1] - o);
  xg[poff[p] + c] = c < n ? x[knots[o + c]] : 0.0;
}

// t_p = C_p^-1 xg_p, one wavefront per row of every part; 16-byte loads of
// the row (rows start 256-byte aligned: npad is a multiple of 32), two
// independent accumulators per lane.
__global__ void __launch_bounds__(kBlock) block_gemv_kernel(
    const int64_t* __restrict__ off, const int32_t* __restrict__ npad, const int64_t* __restrict__ aoff,
    const int64_t* __restrict__ poff, const double* __restrict__ mat, const double* __restrict__ xg,
    double* __restrict__ t, const int* __restrict__ stop) {
  if (stop && *stop) return;
  const int p = blockIdx.y;
  const int r = blockIdx.x * (kBlock / kWave) + (threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int64_t o = off[p];
  const int n = (int)(off[p + 1] - o);
  if (r >= n) return;
  const int np = npad[p];
  const double2* X = reinterpret_cast<const double2*>(mat + aoff[p] + (int64_t)r * 2 * np + np);
  const double2* xv = reinterpret_cast<const double2*>(xg + poff[p]);
  const int h = np / 2;
  double a0 = 0.0, a1 = 0.0;
  int c = lane;
  for (; c + kWave < h; c += 2 * kWave) {
    const double2 u0 = X[c], v0 = xv[c];
    const double2 u1 = X[c + kWave], v1 = xv[c + kWave];
    a0 += u0.x * v0.x + u0.y * v0.y;
    a1 += u1.x * v1.x + u1.y * v1.y;
  }
  if (c < h) {
    const double2 u0 = X[c], v0 = xv[c];
    a0 += u0.x * v0.x + u0.y * v0.y;
  }
  const double acc = wave_sum(a0 + a1);
  if (lane == 0) t[o + r] = acc;
}

// FP32 copy of every C_p^-1 (rows and columns padded to npad, zeros beyond #omega_p).
__global__ void to_f32_kernel(const int32_t* __restrict__ npad, const int64_t* __restrict__ aoff,
                              const int64_t* __restrict__ ioff, const double* __restrict__ mat,
                              float* __restrict__ inv32) {
  const int p = blockIdx.y;
  const int np = npad[p];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)np * np) return;
  const int r = (int)(e / np), c = (int)(e - (int64_t)r * np);
  inv32[ioff[p] + e] = (float)mat[aoff[p] + (int64_t)r * 2 * np + np + c];
}

// t_p = C_p^-1 xg_p from the FP32 inverses: 16-byte loads of four entries,
// products and sums in FP64.
__global__ void __launch_bounds__(kBlock) block_gemv_f32_kernel(
    const int64_t* __restrict__ off, const int32_t* __restrict__ npad, const int64_t* __restrict__ ioff,
    const int64_t* __restrict__ poff, const float* __restrict__ inv32, const double* __restrict__ xg,
    double* __restrict__ t, const int* __restrict__ stop) {
  if (stop && *stop) return;
  const int p = blockIdx.y;
  const int r = blockIdx.x * (kBlock / kWave) + (threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int64_t o = off[p];
  const int n = (int)(off[p + 1] - o);
  if (r >= n) return;
  const int np = npad[p];
  const float4* X = reinterpret_cast<const float4*>(inv32 + ioff[p] + (int64_t)r * np);
  const double2* xv = reinterpret_cast<const double2*>(xg + poff[p]);
  const int q = np / 4;
  double a0 = 0.0, a1 = 0.0;
  for (int c = lane; c < q; c += kWave) {
    const float4 u = X[c];
    const double2 v0 = xv[2 * c], v1 = xv[2 * c + 1];
    a0 += (double)u.x * v0.x + (double)u.y * v0.y;
    a1 += (double)u.z * v1.x + (double)u.w * v1.y;
  }
  const double acc = wave_sum(a0 + a1);
  if (lane == 0) t[o + r] = acc;
}

// y_i = sum over the parts holding knot i (in part order) of D_ii t_p(i).
__global__ void combine_kernel(int64_t N, const int64_t* __restrict__ moff, const int64_t* __restrict__ mslot,
                               const double* __restrict__ t, double* __restrict__ y,
                               const int* __restrict__ stop) {
  if (stop && *stop) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int64_t a = moff[i], b = moff[i + 1];
  const double d = 1.0 / (double)(b - a);
  double s = 0.0;
  for (int64_t k = a; k < b; ++k) s += d * t[mslot[k]];
  y[i] = s;
}

__global__ void __launch_bounds__(kBlock) spmv_kernel(int64_t N, const int64_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ cols,
                                                      const double* __restrict__ val,
                                                      const double* __restrict__ x, double* __restrict__ y,
                                                      const double* __restrict__ sub,
                                                      const int* __restrict__ stop) {
  if (stop && *stop) return;
  const int64_t i = (int64_t)blockIdx.x * (kBlock / kWave) + (threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  if (i >= N) return;
  double acc = 0.0;
  for (int64_t e = rowptr[i] + lane; e < rowptr[i + 1]; e += kWave) acc += val[e] * x[cols[e]];
  acc = wave_sum(acc);
  if (lane == 0) y[i] = sub ? sub[i] - acc : acc;
}

// part[k * kDotBlocks + blk] = partial <w, V_k> over this block's rows, k < nv.
__global__ void __launch_bounds__(kBlock) multidot_kernel(int64_t N, int nv, const double* __restrict__ V,
                                                          const double* __restrict__ w,
                                                          double* __restrict__ part,
                                                          const int* __restrict__ stop) {
  if (stop && *stop) return;
  __shared__ double red[kBlock / kWave];
  const int64_t chunk = (N + kDotBlocks - 1) / kDotBlocks;
  const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = min(N, i0 + chunk);
  for (int k = 0; k < nv; ++k) {
    const double* v = V + (int64_t)k * N;
    double acc = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) acc += w[i] * v[i];
    acc = wave_sum(acc);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int q = 0; q < kBlock / kWave; ++q) s += red[q];
      part[(int64_t)k * kDotBlocks + blockIdx.x] = s;
    }
    __syncthreads();
  }
}

// h[k] (+)= sum of the partials of dot k, in block order; one wavefront per dot.
__global__ void reduce_dots_kernel(int nv, const double* __restrict__ part, double* __restrict__ h, int accumulate,
                                   const int* __restrict__ stop) {
  if (stop && *stop) return;
  const int k = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (k >= nv) return;
  double acc = 0.0;
  for (int b = lane; b < kDotBlocks; b += kWave) acc += part[(int64_t)k * kDotBlocks + b];
  acc = wave_sum(acc);
  if (lane == 0) h[k] = accumulate ? h[k] + acc : acc;
}

// w -= sum_k c[k] V_k  (c read from device memory)
__global__ void update_kernel(int64_t N, int nv, const double* __restrict__ V, const double* __restrict__ c,
                              double* __restrict__ w, const int* __restrict__ stop) {
  if (stop && *stop) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s = w[i];
  for (int k = 0; k < nv; ++k) s -= c[k] * V[(int64_t)k * N + i];
  w[i] = s;
}

// v = w / sqrt(nrm2) (v = 0 when the norm vanishes); nrm[1] receives the norm.
__global__ void normalise_kernel(int64_t N, const double* __restrict__ w, double* __restrict__ nrm,
                                 double* __restrict__ v, const int* __restrict__ stop) {
  if (stop && *stop) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double s = sqrt(nrm[0]);
  if (i == 0) nrm[1] = s;
  if (i < N) v[i] = s > 0.0 ? w[i] / s : 0.0;
}

// s = sum_k y[k] V_k
__global__ void combine_basis_kernel(int64_t N, int nv, const double* __restrict__ V,
                                     const double* __restrict__ y, double* __restrict__ s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double a = 0.0;
  for (int k = 0; k < nv; ++k) a += y[k] * V[(int64_t)k * N + i];
  s[i] = a;
}

__global__ void axpy_kernel(int64_t N, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) y[i] += x[i];
}

__global__ void copy_kernel(int64_t N, const double* __restrict__ x, double* __restrict__ y,
                            const int* __restrict__ stop) {
  if (stop && *stop) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) y[i] = x[i];
}

// GMRES state kept on the device between host checks.
struct GmState {
  int stop;     // the cycle has ended: converged or out of iterations
  int k;        // Arnoldi columns of this cycle
  int iters;    // iterations over all cycles
  int pad;
  double rel;   // |g_{k}| / |r|
};

// Column j of the Hessenberg matrix (row-major, (m+1) x m) from the Gram-
// Schmidt coefficients h[0..j] and the new vector's norm nrm[1]; the earlier
// Givens rotations on it, a new rotation, the residual estimate and the stop
// test.  One thread.
__global__ void givens_kernel(int j, int m, const double* __restrict__ h, const double* __restrict__ nrm,
                              double* __restrict__ Hm, double* __restrict__ cs, double* __restrict__ sn,
                              double* __restrict__ g, GmState* __restrict__ gs, double bnorm, double rtol,
                              int max_iter) {
  if (threadIdx.x != 0 || gs->stop) return;
  for (int i = 0; i <= j; ++i) Hm[(int64_t)i * m + j] = h[i];
  Hm[(int64_t)(j + 1) * m + j] = nrm[1];
  for (int i = 0; i < j; ++i) {
    const double a = Hm[(int64_t)i * m + j], c = Hm[(int64_t)(i + 1) * m + j];
    Hm[(int64_t)i * m + j] = cs[i] * a + sn[i] * c;
    Hm[(int64_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
  }
  const double a = Hm[(int64_t)j * m + j], c = Hm[(int64_t)(j + 1) * m + j];
  const double den = hypot(a, c);
  cs[j] = a / den;
  sn[j] = c / den;
  Hm[(int64_t)j * m + j] = den;
  Hm[(int64_t)(j + 1) * m + j] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  gs->iters += 1;
  gs->k = j + 1;
  gs->rel = fabs(g[j + 1]) / bnorm;
  if (gs->rel <= rtol || gs->iters >= max_iter) gs->stop = 1;
}

inline dim3 grid1(int64_t N) { return dim3((unsigned)std::max<int64_t>(1, (N + kBlock - 1) / kBlock)); }

// Parts of the circles: px slabs by centre x, each split into py parts by
// centre y; stable sorts, so equal coordinates keep circle order.
std::vector<int32_t> circle_parts(const HostCover& H, int px, int py, int32_t& P) {
  const int n = H.nc;
  std::vector<int32_t> part(n, 0), byx(n);
  std::iota(byx.begin(), byx.end(), 0);
  std::stable_sort(byx.begin(), byx.end(), [&](int a, int b) { return H.cx[a] < H.cx[b]; });
  for (int s = 0; s < px; ++s) {
    std::vector<int32_t> slab(byx.begin() + (int64_t)s * n / px, byx.begin() + (int64_t)(s + 1) * n / px);
    std::stable_sort(slab.begin(), slab.end(), [&](int a, int b) { return H.cy[a] < H.cy[b]; });
    const int64_t k = (int64_t)slab.size();
    for (int t = 0; t < py; ++t)
      for (int64_t q = t * k / py; q < (t + 1) * k / py; ++q) part[slab[q]] = s * py + t;
  }
  std::vector<int32_t> renum(px * py, -1);
  for (int m = 0; m < n; ++m) renum[part[m]] = 0;
  P = 0;
  for (auto& r : renum)
    if (r == 0) r = P++;
  for (auto& v : part) v = renum[v];
  return part;
}

struct Ras {
  pdd_ras r;
  hipStream_t st;
  // y = M^-1 x (nothing when *stop is set)
  void apply(const double* x, double* y, const int* stop = nullptr) const {
    hipLaunchKernelGGL(gather_x_kernel, dim3((unsigned)((r->max_npad + kBlock - 1) / kBlock), (unsigned)r->P),
                       dim3(kBlock), 0, st, r->d_off.ptr<int64_t>(), r->d_knots.ptr<int32_t>(),
                       r->d_npad.ptr<int32_t>(), r->d_poff.ptr<int64_t>(), x, r->xg.ptr<double>(), stop);
    const dim3 g((unsigned)((r->max_npad + 3) / 4), (unsigned)r->P);
    if (r->f32)
      hipLaunchKernelGGL(block_gemv_f32_kernel, g, dim3(kBlock), 0, st, r->d_off.ptr<int64_t>(),
                         r->d_npad.ptr<int32_t>(), r->d_ioff.ptr<int64_t>(), r->d_poff.ptr<int64_t>(),
                         r->inv32.ptr<float>(), r->xg.ptr<double>(), r->t.ptr<double>(), stop);
    else
      hipLaunchKernelGGL(block_gemv_kernel, g, dim3(kBlock), 0, st, r->d_off.ptr<int64_t>(),
                         r->d_npad.ptr<int32_t>(), r->d_aoff.ptr<int64_t>(), r->d_poff.ptr<int64_t>(),
                         r->mat.ptr<double>(), r->xg.ptr<double>(), r->t.ptr<double>(), stop);
    const int64_t N = r->sys->cover->H.N();
    hipLaunchKernelGGL(combine_kernel, grid1(N), dim3(kBlock), 0, st, N, r->d_moff.ptr<int64_t>(),
                       r->d_mslot.ptr<int64_t>(), r->t.ptr<double>(), y, stop);
  }
};

}  // namespace

pdd_status ras_build_impl(pdd_system sys, const pdd_ras_opts* opts, hipStream_t st, pdd_ras* out) {
  const int px = opts ? opts->parts_x : 1, py = opts ? opts->parts_y : 1;
  if (px < 1 || py < 1 || (int64_t)px * py > 65535)
    return fail(PDD_EINVAL, "pdd_ras_build: parts_x and parts_y must be >= 1");
  const HostCover& H = sys->cover->H;
  const DeviceCover& D = sys->cover->D;
  const int64_t N = H.N();
  auto R = std::make_unique<pdd_ras_s>();
  R->sys = sys;
  int32_t P = 0;
  const std::vector<int32_t> cpart = circle_parts(H, px, py, P);
  std::vector<int32_t> kpart(N);
  for (int64_t i = 0; i < N; ++i) kpart[i] = cpart[H.owner[i]];
  // omega_p: own knots and one layer of the symmetric graph of C (rows of
  // C and of C^T), built per part from its own knots
  std::vector<int64_t> trp(N + 1, 0);
  for (int64_t e = 0; e < H.rowptr[N]; ++e) ++trp[H.cols[e] + 1];
  for (int64_t i = 0; i < N; ++i) trp[i + 1] += trp[i];
  std::vector<int32_t> trc(H.rowptr[N]);
  {
    std::vector<int64_t> fill(trp.begin(), trp.end() - 1);
    for (int64_t i = 0; i < N; ++i)
      for (int64_t e = H.rowptr[i]; e < H.rowptr[i + 1]; ++e) trc[fill[H.cols[e]]++] = (int32_t)i;
  }
  std::vector<std::vector<int32_t>> own(P);
  for (int64_t i = 0; i < N; ++i) own[kpart[i]].push_back((int32_t)i);
  R->P = P;
  R->off.assign(P + 1, 0);
  std::vector<std::vector<int64_t>> slots(N);
  std::vector<int32_t> w, seen(N, -1);   // seen[j] == p: j already in omega_p
  for (int p = 0; p < P; ++p) {
    w.clear();
    auto add = [&](int32_t j) {
      if (seen[j] != p) {
        seen[j] = p;
        w.push_back(j);
      }
    };
    for (int32_t i : own[p]) {
      add(i);
      for (int64_t e = H.rowptr[i]; e < H.rowptr[i + 1]; ++e) add(H.cols[e]);
      for (int64_t e = trp[i]; e < trp[i + 1]; ++e) add(trc[e]);
    }
    std::sort(w.begin(), w.end());
    for (int32_t i : w) {
      slots[i].push_back((int64_t)R->knots.size());
      R->knots.push_back(i);
    }
    R->off[p + 1] = (int64_t)R->knots.size();
  }
  R->total = (int64_t)R->knots.size();
  R->npad.resize(P);
  R->aoff.assign(P, 0);
  int64_t mat_doubles = 0, work_bytes = 0, piv_total = 0;
  std::vector<int64_t> woff(P), poff(P);
  for (int p = 0; p < P; ++p) {
    const int64_t n = R->off[p + 1] - R->off[p];
    if (n > 4096)
      return fail(PDD_EINVAL, "pdd_ras_build: a part holds " + std::to_string(n) +
                                  " knots with its overlap (at most 4096): use more parts");
    const int np = (int)((n + 31) / 32 * 32);
    R->npad[p] = np;
    R->max_npad = std::max(R->max_npad, np);
    R->aoff[p] = mat_doubles;
    mat_doubles += (int64_t)np * 2 * np;
    woff[p] = work_bytes;
    work_bytes += (int64_t)((lu_work_bytes_per_matrix(np) + 255) / 256 * 256);
    poff[p] = piv_total;
    piv_total += np;
  }
  std::vector<int64_t> moff(N + 1, 0), mslot;
  mslot.reserve(R->total);
  for (int64_t i = 0; i < N; ++i) {
    mslot.insert(mslot.end(), slots[i].begin(), slots[i].end());
    moff[i + 1] = (int64_t)mslot.size();
  }
  slots.clear();
  R->d_off.upload(R->off);
  R->d_knots.upload(R->knots);
  R->d_npad.upload(R->npad);
  R->d_aoff.upload(R->aoff);
  R->poff = poff;
  R->d_poff.upload(R->poff);
  R->xg.alloc(std::max<int64_t>(1, piv_total) * sizeof(double));
  R->d_moff.upload(moff);
  R->d_mslot.upload(mslot);
  R->mat.alloc(mat_doubles * sizeof(double));
  R->piv.alloc(piv_total * sizeof(int32_t));
  R->status.alloc(P * sizeof(int32_t));
  R->work.alloc(work_bytes);
  R->t.alloc(std::max<int64_t>(1, R->total) * sizeof(double));
  PDD_HIP(hipMemsetAsync(R->mat.ptr<void>(), 0, mat_doubles * sizeof(double), st));
  PDD_HIP(hipMemsetAsync(R->status.ptr<void>(), 0, P * sizeof(int32_t), st));
  const dim3 g((unsigned)((R->max_npad + 3) / 4), (unsigned)P);
  hipLaunchKernelGGL(gather_blocks_kernel, g, dim3(kBlock), 0, st, R->d_off.ptr<int64_t>(),
                     R->d_knots.ptr<int32_t>(), R->d_npad.ptr<int32_t>(), R->d_aoff.ptr<int64_t>(),
                     D.rowptr.ptr<int64_t>(), D.cols.ptr<int32_t>(), sys->val.ptr<double>(),
                     R->mat.ptr<double>());
  PDD_HIP(hipGetLastError());
  std::vector<LuItem> its(P);
  char* wb = R->work.ptr<char>();
  for (int p = 0; p < P; ++p) {
    LuItem& it = its[p];
    it.A = R->mat.ptr<double>() + R->aoff[p];
    it.piv = R->piv.ptr<int32_t>() + poff[p];
    it.status = R->status.ptr<int32_t>() + p;
    it.work = reinterpret_cast<LuWork*>(wb + woff[p]);
    it.uinv = reinterpret_cast<double*>(wb + woff[p] + lu_work_header_bytes());
    it.n = R->npad[p];
    it.ld = 2 * R->npad[p];
    it.nrhs = R->npad[p];
    it.cls = lu_panel_class(it.n);
  }
  {
    LuPlan plan;
    plan.build(its);
    plan.launch(st, 1 << 30);
    PDD_HIP(hipGetLastError());
    PDD_HIP(hipStreamSynchronize(st));   // the plan's device lists are freed on return
  }
  std::vector<int32_t> stat(P);
  PDD_HIP(hipMemcpy(stat.data(), R->status.ptr<void>(), P * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int p = 0; p < P; ++p)
    if (stat[p]) return fail(PDD_EBREAKDOWN, "pdd_ras_build: zero pivot in block " + std::to_string(p));
  if (opts && opts->fp32_inverses) {
    R->f32 = true;
    R->ioff.assign(P, 0);
    int64_t nf = 0;
    for (int p = 0; p < P; ++p) {
      R->ioff[p] = nf;
      nf += (int64_t)R->npad[p] * R->npad[p];
    }
    R->d_ioff.upload(R->ioff);
    R->inv32.alloc(nf * sizeof(float));
    const int64_t most = (int64_t)R->max_npad * R->max_npad;
    hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)((most + kBlock - 1) / kBlock), (unsigned)P), dim3(kBlock),
                       0, st, R->d_npad.ptr<int32_t>(), R->d_aoff.ptr<int64_t>(), R->d_ioff.ptr<int64_t>(),
                       R->mat.ptr<double>(), R->inv32.ptr<float>());
    PDD_HIP(hipGetLastError());
    PDD_HIP(hipStreamSynchronize(st));
    R->mat.release();                    // the FP64 factors are no longer needed
  }
  *out = R.release();
  return PDD_OK;
}

pdd_status gmres_impl(pdd_system sys, pdd_ras ras, const double* rhs, double* u, const pdd_gmres_opts* opts,
                      hipStream_t st, pdd_solve_info* info) {
  const HostCover& H = sys->cover->H;
  const DeviceCover& D = sys->cover->D;
  const int64_t N = H.N();
  const double rtol = (opts && opts->rtol > 0.0) ? opts->rtol : 1e-12;
  const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 2000;
  const int m = (opts && opts->restart > 0) ? std::min(opts->restart, 200) : 30;
  const double* b = rhs ? rhs : sys->b.ptr<double>();
  // V [m+1][N], w, z, s, partial sums, h, y, norm scratch, Hessenberg
  // [(m+1) m], rotations, g, state
  const int64_t nv = (int64_t)(m + 1) * N;
  const int64_t nd = nv + 3 * N + (int64_t)(m + 2) * kDotBlocks + 2 * (m + 2) + 4 + (int64_t)(m + 1) * m +
                     2 * m + (m + 1);
  DevBuf work;
  work.alloc(sizeof(double) * nd + sizeof(GmState));
  double* V = work.ptr<double>();
  double* w = V + nv;
  double* z = w + N;
  double* s = z + N;
  double* part = s + N;
  double* h = part + (int64_t)(m + 2) * kDotBlocks;
  double* yv = h + (m + 2);
  double* nrm = yv + (m + 2);
  double* Hm = nrm + 4;
  double* cs = Hm + (int64_t)(m + 1) * m;
  double* sn = cs + m;
  double* g = sn + m;
  GmState* gs = reinterpret_cast<GmState*>(g + (m + 1));
  const int* stop = &gs->stop;
  const Ras prec{ras, st};
  auto precond = [&](const double* x, double* y, const int* flag) {
    if (ras) prec.apply(x, y, flag);
    else hipLaunchKernelGGL(copy_kernel, grid1(N), dim3(kBlock), 0, st, N, x, y, flag);
  };
  auto spmv = [&](const double* x, double* y, const double* sub, const int* flag) {
    hipLaunchKernelGGL(spmv_kernel, dim3((unsigned)std::max<int64_t>(1, (N + 3) / 4)), dim3(kBlock), 0, st, N,
                       D.rowptr.ptr<int64_t>(), D.cols.ptr<int32_t>(), sys->val.ptr<double>(), x, y, sub, flag);
  };
  auto dots = [&](int k, const double* Vb, const double* x, double* out, int acc, const int* flag) {
    hipLaunchKernelGGL(multidot_kernel, dim3(kDotBlocks), dim3(kBlock), 0, st, N, k, Vb, x, part, flag);
    hipLaunchKernelGGL(reduce_dots_kernel, dim3((unsigned)((k + 3) / 4)), dim3(kBlock), 0, st, k, part, out, acc,
                       flag);
  };
  auto norm_into = [&](const double* x, double* v, const int* flag) {   // v = x / |x|, nrm[1] = |x|
    dots(1, x, x, nrm, 0, flag);
    hipLaunchKernelGGL(normalise_kernel, grid1(N), dim3(kBlock), 0, st, N, x, nrm, v, flag);
  };
  auto read = [&](const void* d, void* hst, size_t bytes) {
    PDD_HIP(hipMemcpyAsync(hst, d, bytes, hipMemcpyDeviceToHost, st));
    PDD_HIP(hipStreamSynchronize(st));
  };
  double bn2 = 0.0;
  dots(1, b, b, nrm, 0, nullptr);
  read(nrm, &bn2, sizeof(double));
  const double bnorm = std::sqrt(bn2);
  PDD_HIP(hipMemsetAsync(u, 0, N * sizeof(double), st));
  pdd_solve_info res{0, 0, 0.0};
  if (bnorm == 0.0) {
    PDD_HIP(hipStreamSynchronize(st));
    res.converged = 1;
    if (info) *info = res;
    return PDD_OK;
  }
  // Iterations are enqueued in batches; the host reads the device state once
  // per batch (kernels of iterations past the stop return at once).
  constexpr int kBatch = 8;
  std::vector<double> Hh((size_t)(m + 1) * m), gh(m + 1);
  int it = 0;
  double rel = 1.0;
  GmState hs{};
  while (it < max_iter) {
    spmv(u, w, b, nullptr);              // w = b - C u
    double nb[2];
    norm_into(w, V, nullptr);
    read(nrm, nb, 2 * sizeof(double));
    rel = nb[1] / bnorm;
    if (rel <= rtol) break;
    std::vector<double> g0(m + 1, 0.0);
    g0[0] = nb[1];
    GmState init{0, 0, it, 0, rel};
    PDD_HIP(hipMemcpyAsync(g, g0.data(), (m + 1) * sizeof(double), hipMemcpyHostToDevice, st));
    PDD_HIP(hipMemcpyAsync(gs, &init, sizeof(GmState), hipMemcpyHostToDevice, st));
    for (int j0 = 0; j0 < m; j0 += kBatch) {
      const int j1 = std::min(m, j0 + kBatch);
      for (int j = j0; j < j1; ++j) {
        precond(V + (int64_t)j * N, z, stop);
        spmv(z, w, nullptr, stop);
        // classical Gram-Schmidt, twice: h = V^T w, w -= V h; c = V^T w,
        // w -= V c, h += c (the second reduction re-sums the same partials)
        dots(j + 1, V, w, h, 0, stop);
        hipLaunchKernelGGL(update_kernel, grid1(N), dim3(kBlock), 0, st, N, j + 1, V, h, w, stop);
        dots(j + 1, V, w, yv, 0, stop);
        hipLaunchKernelGGL(update_kernel, grid1(N), dim3(kBlock), 0, st, N, j + 1, V, yv, w, stop);
        hipLaunchKernelGGL(reduce_dots_kernel, dim3((unsigned)((j + 1 + 3) / 4)), dim3(kBlock), 0, st, j + 1,
                           part, h, 1, stop);
        norm_into(w, V + (int64_t)(j + 1) * N, stop);
        hipLaunchKernelGGL(givens_kernel, dim3(1), dim3(64), 0, st, j, m, h, nrm, Hm, cs, sn, g, gs, bnorm,
                           rtol, max_iter);
      }
      PDD_HIP(hipGetLastError());
      read(gs, &hs, sizeof(GmState));
      if (hs.stop) break;
    }
    const int k = hs.k;
    it = hs.iters;
    rel = hs.rel;
    // y = H_k^-1 g_k (upper triangular after the rotations), u += M^-1 (V_k y)
    read(Hm, Hh.data(), (size_t)(m + 1) * m * sizeof(double));
    read(g, gh.data(), (m + 1) * sizeof(double));
    std::vector<double> y(std::max(k, 1));
    for (int i = k - 1; i >= 0; --i) {
      double t = gh[i];
      for (int q = i + 1; q < k; ++q) t -= Hh[(size_t)i * m + q] * y[q];
      y[i] = t / Hh[(size_t)i * m + i];
    }
    if (k > 0) {
      PDD_HIP(hipMemcpyAsync(yv, y.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(combine_basis_kernel, grid1(N), dim3(kBlock), 0, st, N, k, V, yv, s);
      precond(s, z, nullptr);
      hipLaunchKernelGGL(axpy_kernel, grid1(N), dim3(kBlock), 0, st, N, z, u);
      PDD_HIP(hipGetLastError());
    }
    PDD_HIP(hipStreamSynchronize(st));   // y lives on the host stack
    if (rel <= rtol || k == 0) break;
  }
  PDD_HIP(hipStreamSynchronize(st));
  res.iterations = it;
  res.converged = rel <= rtol ? 1 : 0;
  res.rel_residual = rel;
  if (info) *info = res;
  if (!res.converged) return fail(PDD_ENOCONV, "pdd_solve_gmres: no convergence");
  return PDD_OK;
}

}  // namespace pdd

using namespace pdd;

extern "C" {

pdd_status pdd_ras_build(pdd_system sys, const pdd_ras_opts* opts, void* stream, pdd_ras* out) {
  if (!sys || !out) return fail(PDD_EINVAL, "pdd_ras_build: null argument");
  *out = nullptr;
  try {
    return ras_build_impl(sys, opts, (hipStream_t)stream, out);
  } catch (const HipError& e) {
    return fail(e.code == hipErrorOutOfMemory ? PDD_ENOMEM : PDD_EDEVICE, e.what());
  } catch (const std::bad_alloc&) {
    return fail(PDD_ENOMEM, "pdd_ras_build: out of host memory");
  } catch (const std::exception& e) {
    return fail(PDD_EDEVICE, std::string("pdd_ras_build: ") + e.what());
  }
}

pdd_status pdd_ras_get_parts(pdd_ras ras, int32_t* n_parts, int64_t* omega_off, int32_t* omega) {
  if (!ras) return fail(PDD_EINVAL, "pdd_ras_get_parts: null handle");
  if (n_parts) *n_parts = ras->P;
  if (omega_off) std::copy(ras->off.begin(), ras->off.end(), omega_off);
  if (omega) std::copy(ras->knots.begin(), ras->knots.end(), omega);
  return PDD_OK;
}

pdd_status pdd_ras_apply(pdd_ras ras, const double* x, double* y, void* stream) {
  if (!ras || !x || !y) return fail(PDD_EINVAL, "pdd_ras_apply: null argument");
  try {
    const Ras prec{ras, (hipStream_t)stream};
    prec.apply(x, y, nullptr);
    PDD_HIP(hipGetLastError());
    return PDD_OK;
  } catch (const HipError& e) {
    return fail(PDD_EDEVICE, e.what());
  }
}

pdd_status pdd_solve_gmres(pdd_system sys, pdd_ras ras, const double* rhs, double* u,
                           const pdd_gmres_opts* opts, void* stream, pdd_solve_info* info) {
  if (!sys || !u) return fail(PDD_EINVAL, "pdd_solve_gmres: null argument");
  if (ras && ras->sys != sys) return fail(PDD_EINVAL, "pdd_solve_gmres: preconditioner of another system");
  try {
    return gmres_impl(sys, ras, rhs, u, opts, (hipStream_t)stream, info);
  } catch (const HipError& e) {
    return fail(e.code == hipErrorOutOfMemory ? PDD_ENOMEM : PDD_EDEVICE, e.what());
  } catch (const std::bad_alloc&) {
    return fail(PDD_ENOMEM, "pdd_solve_gmres: out of host memory");
  } catch (const std::exception& e) {
    return fail(PDD_EDEVICE, std::string("pdd_solve_gmres: ") + e.what());
  }
}

void pdd_destroy_ras(pdd_ras ras) { delete ras; }

}  // extern "C"
