// Batched LU with partial pivoting of the per-circle collocation matrices and
// solution of the right-hand sides (Section 3.3, eqs. 40-41; the paper uses
// one QR factorisation per circle, here LU with partial pivoting).
//
// One workgroup (8 wavefronts) owns one matrix [A_II | R] (n x ld, row-major).
// Two-level right-looking factorisation:
//   * outer panels of kOuter = 128 columns;
//   * each outer panel is factorised by sub-panels of NBI columns held in
//     registers (thread t owns rows k0 + t + 512 s), column by column with a
//     workgroup-wide pivot search; the sub-panel's interchanges, its block row
//     of U and the update of the rest of the outer panel follow;
//   * the outer panel's interchanges are applied to all other columns, its
//     block row of U is formed by a blocked triangular solve, and the trailing
//     matrix -- including the right-hand-side columns, which are thereby
//     eliminated forward -- is updated with K = 128.
// Back substitution U W = R' then runs right-looking from the bottom in
// 128-row blocks.  Every rectangular update A[r, c] -= A[r, k] A[k, c] goes
// through one FP64 MFMA routine (v_mfma_f64_16x16x4: A[i][k] in lane i + 16 k,
// B[k][j] in lane j + 16 k, D[i][j] in register i / 4 of lane j + 16 (i mod 4))
// with 128 x 128 workgroup tiles and K streamed through LDS in chunks of 32,
// the next chunk's global loads issued before the current chunk's MFMAs.
#include "kernels.h"

namespace pdd {

namespace {

constexpr int kThreads = 512;
constexpr int kOuter = 128;
constexpr int kGT = 128;        // update tile (rows and columns)
constexpr int kGK = 32;         // K chunk
constexpr int kPad = 1;
constexpr int kWave = 64;

typedef double dbl4 __attribute__((ext_vector_type(4)));

struct GemmLds {
  double Lt[kGK][kGT + kPad];   // -A[r, k] chunk, transposed
  double Ut[kGK][kGT + kPad];   //  A[k, c] chunk
};

// A[r0:r1, c0:c1] -= A[r0:r1, k0:k1] A[k0:k1, c0:c1]; the three blocks are
// disjoint.  Called by all threads of the workgroup; ends with a barrier.
// Addresses are one per-lane base pointer plus workgroup-uniform offsets, and
// the edge tests are per-lane bit masks, to keep register use low.
__device__ __attribute__((always_inline)) void gemm_sub(double* __restrict__ A, int ld, int r0, int r1, int c0, int c1,
                                                         int k0, int k1, GemmLds& s) {
  // element offsets from A fit in 32 bits (n * ld < 2^31)
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;       // 4 x 2 wavefronts: 32 rows x 64 columns each
  const int li = lane & 15, lk = lane >> 4;
  const int lrow = tid >> 5, lcol = tid & 31;      // operand loads: A[r, k] chunk
  const int urow = tid >> 7, ucol = tid & 127;     //                A[k, c] chunk
  double* __restrict__ lt_st = &s.Lt[lcol][lrow];
  double* __restrict__ ut_st = &s.Ut[urow][ucol];
  const double* __restrict__ lt_rd = &s.Lt[lk][32 * wr + li];
  const double* __restrict__ ut_rd = &s.Ut[lk][64 * wc + li];
#pragma unroll 1
  for (int rt = r0; rt < r1; rt += kGT) {
#pragma unroll 1
    for (int ct = c0; ct < c1; ct += kGT) {
      const int crow = rt + 32 * wr + lk, ccol = ct + 64 * wc + li;
      const int coff = crow * ld + ccol;
      unsigned rmask = 0, cmask = 0;
#pragma unroll
      for (int t = 0; t < 8; ++t)        // t = 4 bi + v: row offset 16 bi + 4 v
        rmask |= (crow + 16 * (t >> 2) + 4 * (t & 3) < r1) ? (1u << t) : 0u;
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) cmask |= (ccol + 16 * bj < c1) ? (1u << bj) : 0u;
      dbl4 acc[2][4];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int bj = 0; bj < 4; ++bj) {
            const bool ok = ((rmask >> (4 * bi + v)) & (cmask >> bj) & 1u) != 0;
            const double cv = A[ok ? coff + (16 * bi + 4 * v) * ld + 16 * bj : 0];
            acc[bi][bj][v] = ok ? cv : 0.0;
          }
      const int loff = (rt + lrow) * ld + lcol;
      const int uoff = urow * ld + ct + ucol;
      unsigned lmask = 0;
#pragma unroll
      for (int it = 0; it < 8; ++it) lmask |= (rt + lrow + 16 * it < r1) ? (1u << it) : 0u;
      const bool ucol_ok = ct + ucol < c1;
      double pl[8], pu[8];
      // out-of-range elements read A[0] (always valid) and are then zeroed
      auto fetch = [&](int kc) {
        const bool lk_ok = kc + lcol < k1;
#pragma unroll
        for (int it = 0; it < 8; ++it) {
          const bool okl = lk_ok && ((lmask >> it) & 1u);
          const bool oku = ucol_ok && kc + urow + 4 * it < k1;
          const double vl = A[okl ? loff + 16 * it * ld + kc : 0];
          const double vu = A[oku ? uoff + (kc + 4 * it) * ld : 0];
          pl[it] = okl ? vl : 0.0;
          pu[it] = oku ? vu : 0.0;
        }
      };
      fetch(k0);
#pragma unroll 1
      for (int kc = k0; kc < k1; kc += kGK) {
#pragma unroll
        for (int it = 0; it < 8; ++it) {
          lt_st[16 * it] = -pl[it];
          ut_st[4 * it * (kGT + kPad)] = pu[it];
        }
        __syncthreads();
        if (kc + kGK < k1) fetch(kc + kGK);
#pragma unroll
        for (int ks = 0; ks < kGK / 4; ++ks) {
          double a[2], b[4];
#pragma unroll
          for (int bi = 0; bi < 2; ++bi) a[bi] = lt_rd[4 * ks * (kGT + kPad) + 16 * bi];
#pragma unroll
          for (int bj = 0; bj < 4; ++bj) b[bj] = ut_rd[4 * ks * (kGT + kPad) + 16 * bj];
#pragma unroll
          for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
              acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
        }
        __syncthreads();
      }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int bj = 0; bj < 4; ++bj) {
            const bool ok = ((rmask >> (4 * bi + v)) & (cmask >> bj) & 1u) != 0;
            if (ok) A[coff + (16 * bi + 4 * v) * ld + 16 * bj] = acc[bi][bj][v];
          }
    }
  }
  __syncthreads();
}

// Rows [a, a+w) of columns [c0, c1) <- L^-1 (rows), L = unit lower triangle of
// A[a:a+w, a:a+w] (w <= NB).  Ends with a barrier.
template <int NB>
__device__ __noinline__ void trsm_rows(double* __restrict__ A, int ld, int a, int w, int c0, int c1,
                          double (*sL)[NB + 1]) {
  const int tid = threadIdx.x;
  for (int idx = tid; idx < NB * NB; idx += kThreads) {
    const int i = idx / NB, j = idx - i * NB;
    sL[i][j] = (i < w && j < w) ? A[(int64_t)(a + i) * ld + a + j] : 0.0;
  }
  __syncthreads();
  for (int col = c0 + tid; col < c1; col += kThreads) {
    double x[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) x[c] = (c < w) ? A[(int64_t)(a + c) * ld + col] : 0.0;
#pragma unroll 1
    for (int c = 1; c < w; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int c2 = 0; c2 < NB; ++c2) acc += (c2 < c) ? sL[c][c2] * x[c2] : 0.0;
#pragma unroll
      for (int c3 = 0; c3 < NB; ++c3) x[c3] = (c3 == c) ? x[c3] - acc : x[c3];
    }
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < w) A[(int64_t)(a + c) * ld + col] = x[c];
  }
  __syncthreads();
}

// Applies the interchanges (base + t) <-> piv[t], t = 0..cnt-1 in order
// (cnt <= 128), to columns [lo, hi) except [skip0, skip1), as one row
// permutation: thread 0 composes the interchanges over the touched rows (at
// most 2 cnt), then the touched rows are staged through LDS in blocks of 32
// columns and written back permuted.  Ends with a barrier.
struct PermLds {
  int rows[256];      // touched row ids: [base, base + cnt) then the extra rows
  int src[256];       // slot whose (old) contents end up in this slot's row
  int count;
};

__device__ __noinline__ void permute_rows(double* __restrict__ A, int ld, const int* __restrict__ piv,
                                          int base, int cnt, int lo, int hi, int skip0, int skip1,
                                          PermLds& pl, double* __restrict__ scratch) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    int nt = cnt;
    int* cont = pl.src;   // slot of the original row whose contents sit in each slot
    for (int t = 0; t < cnt; ++t) {
      pl.rows[t] = base + t;
      cont[t] = t;
    }
    for (int t = 0; t < cnt; ++t) {
      const int b = piv[t];
      if (b == base + t) continue;
      int sb;
      if (b < base + cnt) {
        sb = b - base;
      } else {
        sb = -1;
        for (int e = cnt; e < nt; ++e)
          if (pl.rows[e] == b) { sb = e; break; }
        if (sb < 0) {
          sb = nt++;
          pl.rows[sb] = b;
          cont[sb] = sb;
        }
      }
      const int tmp = cont[t];
      cont[t] = cont[sb];
      cont[sb] = tmp;
    }
    pl.count = nt;
  }
  __syncthreads();
  const int nt = pl.count;
  for (int c0 = lo; c0 < hi; c0 += 32) {
    const bool skip_block = (c0 >= skip0 && c0 + 32 <= skip1);
    if (!skip_block) {
      for (int idx = tid; idx < nt * 32; idx += kThreads) {
        const int e = idx >> 5, c = c0 + (idx & 31);
        if (c < hi && !(c >= skip0 && c < skip1)) scratch[idx] = A[(int64_t)pl.rows[e] * ld + c];
      }
    }
    __syncthreads();
    if (!skip_block) {
      for (int idx = tid; idx < nt * 32; idx += kThreads) {
        const int e = idx >> 5, cc = idx & 31, c = c0 + cc;
        if (c < hi && !(c >= skip0 && c < skip1))
          A[(int64_t)pl.rows[e] * ld + c] = scratch[(pl.src[e] << 5) + cc];
      }
    }
    __syncthreads();
  }
}

// Rows [a, a+w) of columns [c0, c1) <- U^-1 (rows), U = upper triangle of
// A[a:a+w, a:a+w] with its diagonal (w <= NB).  Ends with a barrier.
template <int NB>
__device__ __noinline__ void trsm_upper_rows(double* __restrict__ A, int ld, int a, int w, int c0,
                                             int c1, double (*sU)[NB + 1]) {
  const int tid = threadIdx.x;
  for (int idx = tid; idx < NB * NB; idx += kThreads) {
    const int i = idx / NB, j = idx - i * NB;
    sU[i][j] = (i < w && j < w) ? A[(int64_t)(a + i) * ld + a + j] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int col = c0 + tid; col < c1; col += kThreads) {
    double x[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) x[c] = (c < w) ? A[(int64_t)(a + c) * ld + col] : 0.0;
#pragma unroll 1
    for (int c = w - 1; c >= 0; --c) {
      double acc = 0.0, xc = 0.0;
#pragma unroll
      for (int c2 = 0; c2 < NB; ++c2) {
        acc += (c2 > c) ? sU[c][c2] * x[c2] : 0.0;
        xc = (c2 == c) ? x[c2] : xc;
      }
      const double v = (xc - acc) / sU[c][c];
#pragma unroll
      for (int c3 = 0; c3 < NB; ++c3) x[c3] = (c3 == c) ? v : x[c3];
    }
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < w) A[(int64_t)(a + c) * ld + col] = x[c];
  }
  __syncthreads();
}

template <int ROWS, int NB>
__global__ __launch_bounds__(kThreads) void lu_solve_kernel(double* __restrict__ A0, int n, int ld,
                                                            int nrhs, int64_t stride,
                                                            int32_t* __restrict__ piv0,
                                                            int32_t* __restrict__ status) {
  __shared__ GemmLds g;
  __shared__ double s_prow[NB], s_krow[NB];
  __shared__ double s_L[NB][NB + 1];
  __shared__ double s_redv[kThreads / 64];
  __shared__ int s_redi[kThreads / 64];
  __shared__ int s_piv[kOuter];
  __shared__ PermLds s_perm;

  double* A = A0 + (int64_t)blockIdx.x * stride;
  int32_t* piv = piv0 + (int64_t)blockIdx.x * n;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int singular = 0;

  for (int K0 = 0; K0 < n; K0 += kOuter) {
    const int kb = min(kOuter, n - K0);
    for (int k0 = K0; k0 < K0 + kb; k0 += NB) {
      const int pw = min(NB, K0 + kb - k0);
      // ---- sub-panel in registers
      double P[ROWS][NB];
#pragma unroll
      for (int s = 0; s < ROWS; ++s) {
        const int row = k0 + tid + kThreads * s;
#pragma unroll
        for (int c = 0; c < NB; ++c)
          P[s][c] = (row < n && c < pw) ? A[(int64_t)row * ld + k0 + c] : 0.0;
      }
#pragma unroll 1
      for (int c = 0; c < pw; ++c) {
        const int kk = k0 + c;
        double colv[ROWS];
#pragma unroll
        for (int s = 0; s < ROWS; ++s) {
          double v = 0.0;
#pragma unroll
          for (int cc = 0; cc < NB; ++cc) v = (cc == c) ? P[s][cc] : v;
          colv[s] = v;
        }
        double bv = -1.0;
        int bi = 0x7fffffff;
#pragma unroll
        for (int s = 0; s < ROWS; ++s) {
          const int row = k0 + tid + kThreads * s;
          const double v = fabs(colv[s]);
          if (row >= kk && row < n && v > bv) { bv = v; bi = row; }
        }
        for (int off = 32; off > 0; off >>= 1) {
          const double ov = __shfl_xor(bv, off, kWave);
          const int oi = __shfl_xor(bi, off, kWave);
          if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (lane == 0) { s_redv[w] = bv; s_redi[w] = bi; }
        __syncthreads();
        bv = s_redv[0];
        bi = s_redi[0];
        for (int t = 1; t < kThreads / 64; ++t) {
          const double ov = s_redv[t];
          const int oi = s_redi[t];
          if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        const int p = (bv > 0.0) ? bi : kk;
        if (!(bv > 0.0)) singular = 1;
        const int tp = (p - k0) & (kThreads - 1), sp = (p - k0) / kThreads;
        if (tid == tp) {
#pragma unroll
          for (int s = 0; s < ROWS; ++s)
            if (s == sp)
#pragma unroll
              for (int cc = 0; cc < NB; ++cc) s_prow[cc] = P[s][cc];
        }
        if (tid == c) {
#pragma unroll
          for (int cc = 0; cc < NB; ++cc) s_krow[cc] = P[0][cc];
        }
        __syncthreads();
        if (tid == c) {
#pragma unroll
          for (int cc = 0; cc < NB; ++cc) P[0][cc] = s_prow[cc];
        }
        if (tid == tp && p != kk) {
#pragma unroll
          for (int s = 0; s < ROWS; ++s)
            if (s == sp)
#pragma unroll
              for (int cc = 0; cc < NB; ++cc) P[s][cc] = s_krow[cc];
        }
        const double pv = s_prow[c];
        if (pv != 0.0) {
          const double inv = 1.0 / pv;
#pragma unroll
          for (int s = 0; s < ROWS; ++s) {
            const int row = k0 + tid + kThreads * s;
            if (row > kk && row < n) {
              double lv = 0.0;
#pragma unroll
              for (int cc = 0; cc < NB; ++cc) lv = (cc == c) ? P[s][cc] : lv;
              lv *= inv;
#pragma unroll
              for (int cc = 0; cc < NB; ++cc) {
                const double upd = P[s][cc] - lv * s_prow[cc];
                P[s][cc] = (cc == c) ? lv : ((cc > c) ? upd : P[s][cc]);
              }
            }
          }
        }
        if (tid == 0) {
          s_piv[kk - K0] = p;
          piv[kk] = p;
        }
        __syncthreads();
      }
#pragma unroll
      for (int s = 0; s < ROWS; ++s) {
        const int row = k0 + tid + kThreads * s;
        if (row < n)
#pragma unroll
          for (int c = 0; c < NB; ++c)
            if (c < pw) A[(int64_t)row * ld + k0 + c] = P[s][c];
      }
      // ---- the sub-panel's interchanges on the rest of the outer panel
      __syncthreads();
      permute_rows(A, ld, s_piv + (k0 - K0), k0, pw, K0, K0 + kb, k0, k0 + pw, s_perm, &g.Lt[0][0]);
      if (k0 + pw < K0 + kb) {
        trsm_rows<NB>(A, ld, k0, pw, k0 + pw, K0 + kb, s_L);
        gemm_sub(A, ld, k0 + pw, n, k0 + pw, K0 + kb, k0, k0 + pw, g);
      }
    }
    // ---- the outer panel's interchanges on every other column
    permute_rows(A, ld, s_piv, K0, kb, 0, ld, K0, K0 + kb, s_perm, &g.Lt[0][0]);
    // ---- block row of U (blocked triangular solve), then the trailing update
    if (K0 + kb < ld) {
      for (int a = K0; a < K0 + kb; a += NB) {
        const int wa = min(NB, K0 + kb - a);
        trsm_rows<NB>(A, ld, a, wa, K0 + kb, ld, s_L);
        if (a + wa < K0 + kb) gemm_sub(A, ld, a + wa, K0 + kb, K0 + kb, ld, a, a + wa, g);
      }
      if (K0 + kb < n) gemm_sub(A, ld, K0 + kb, n, K0 + kb, ld, K0, K0 + kb, g);
    }
  }

  // ---- back substitution U W = R' on columns [n, n + nrhs): 128-row blocks
  //      from the bottom, each solved by 32-row triangles and MFMA updates
  for (int k1 = n; k1 > 0; k1 -= kOuter) {
    const int k0 = max(0, k1 - kOuter);
    for (int b1 = k1; b1 > k0; b1 -= NB) {
      const int a0 = max(k0, b1 - NB);
      trsm_upper_rows<NB>(A, ld, a0, b1 - a0, n, n + nrhs, s_L);
      if (a0 > k0) gemm_sub(A, ld, k0, a0, n, n + nrhs, a0, b1, g);
    }
    if (k0 > 0) gemm_sub(A, ld, 0, k0, n, n + nrhs, k0, k1, g);
  }
  if (tid == 0) status[blockIdx.x] = singular;
}

}  // namespace

void launch_lu_solve(const BucketTables& T, int32_t count, double* A, int64_t mat_stride,
                     int32_t* piv, int32_t* status, hipStream_t st) {
  const int n = T.n;
  if (n <= 512)
    hipLaunchKernelGGL((lu_solve_kernel<1, 32>), dim3(count), dim3(kThreads), 0, st, A, n, T.ld,
                       T.nrhs, mat_stride, piv, status);
  else if (n <= 1024)
    hipLaunchKernelGGL((lu_solve_kernel<2, 32>), dim3(count), dim3(kThreads), 0, st, A, n, T.ld,
                       T.nrhs, mat_stride, piv, status);
  else if (n <= 2048)
    hipLaunchKernelGGL((lu_solve_kernel<4, 16>), dim3(count), dim3(kThreads), 0, st, A, n, T.ld,
                       T.nrhs, mat_stride, piv, status);
  else
    hipLaunchKernelGGL((lu_solve_kernel<8, 8>), dim3(count), dim3(kThreads), 0, st, A, n, T.ld,
                       T.nrhs, mat_stride, piv, status);
}

}  // namespace pdd
