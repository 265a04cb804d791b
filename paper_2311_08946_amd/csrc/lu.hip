// Batched LU with partial pivoting of the per-circle collocation matrices and
// solution of the right-hand sides (Section 3.3, eqs. 40-41; the paper uses
// one QR factorisation per circle, here LU with partial pivoting).
//
// Each matrix is the augmented array [A_II | R] (n x ld, row-major, R in
// columns n .. n + nrhs).  Blocked factorisation in steps of kOuter = 128
// columns (the first one shorter when n is not a multiple of 128),
// left-looking (Crout order: the trailing matrix is never updated as a
// whole; each block is brought up to date with one long-K product when it is
// reached), four launches per step over the whole batch:
//   * lu_pupd_kernel (one workgroup per matrix and 128-row tile of the
//     panel): A[K0:n, K0:K0+128] -= L[K0:n, 0:K0] U[0:K0, K0:K0+128];
//   * lu_panel_own_kernel (one workgroup per matrix, a thread per panel row;
//     orders up to 1024): factorises the step's panel without moving rows --
//     each thread keeps its row and tracks the row's position in the pivoted
//     order -- in groups of 32 columns held in registers, column by column
//     with a workgroup-wide pivot search, then the group's U12 rows and the
//     MFMA update of the rest of the panel; the rows that moved are written
//     to their positions once at the end.  It stores the step's composed row
//     permutation and the inverses of the 32 x 32 diagonal blocks of L11 and
//     U11 in a per-matrix work area, and moves the left part (L) of the rows
//     that moved.  Larger orders use lu_panel_wide_kernel (sub-panels of NB
//     columns in registers, thread t owning rows k0 + t + 512 s, interchanges
//     applied after each sub-panel);
//   * lu_urow_kernel<LEFT> (one workgroup per matrix): forms L11^-1 from the
//     inverses of its 32 x 32 diagonal blocks; after a wide panel, one more
//     workgroup per 128-column tile left of the panel applies the step's
//     interchanges to L;
//   * lu_urow_kernel (one workgroup per matrix and 128-column tile right of
//     the panel): applies the step's interchanges to the tile, brings rows
//     [K0, K0 + kb) up to date with one long-K product and forms
//     U12 = L11^-1 A12 with a second MFMA product -- the right-hand-side
//     columns are among these tiles and are thereby eliminated forward.
// Look-ahead: the first U-row tile of step s (the columns of panel s + 1) is a
// launch of its own; the remaining tiles run on a second stream beside the
// pre-update, panel and interchanges of step s + 1, which touch other
// columns (the interchange record and L11^-1 are kept per step parity).
// The back substitution U W = R' then runs from the bottom in 128-row blocks,
// left-looking: lu_bupd_kernel brings a block's right-hand sides up to date
// with every solved block below it in one long-K product, then
// lu_bdiag_kernel solves the diagonal block (32-row triangles through the
// inverses of U's diagonal blocks, stored by the panel kernel, and MFMA
// updates).
// Every rectangular update A[r, c] -= A[r, k] A[k, c] goes through one FP64
// MFMA routine (v_mfma_f64_16x16x4: A[i][k] in lane i + 16 k, B[k][j] in
// lane j + 16 k, D[i][j] in register i / 4 of lane j + 16 (i mod 4)) with
// 128 x 128 workgroup tiles and K streamed through LDS in chunks of 32, the
// next chunk's global loads issued before the current chunk's MFMAs.
#include <algorithm>
#include <utility>
#include <vector>

#include "runtime.h"

namespace pdd {

namespace {

constexpr int kThreads = 512;
constexpr int kGemmThreads = 256;  // the tiled product launches (pre-update, U rows, back updates)
constexpr int kOuter = 128;
constexpr int kGT = 128;        // update tile (rows and columns)
constexpr int kGK = 32;         // K chunk
constexpr int kPad = 1;
constexpr int kWave = 64;
constexpr int kTB = 32;         // triangular block

// Step boundaries.  Step 0 takes the remainder of n modulo 128 (rounded up
// to a multiple of the 32-column group), every later step 128 columns; a
// multiple of 128 gives plain 128-column steps.  With the short step first,
// the tallest panel (all n rows) is also the narrowest, every later panel has
// at most n - lead rows, and the row tiles of the pre-update are whole.
__host__ __device__ __forceinline__ int lu_lead(int n) {
  const int r = n % kOuter;
  return r == 0 ? kOuter : (r + kTB - 1) / kTB * kTB;
}
__host__ __device__ __forceinline__ int lu_steps(int n) { return (n + kOuter - 1) / kOuter; }
// first column of step s
__host__ __device__ __forceinline__ int lu_k0(int n, int s) {
  const int k = s == 0 ? 0 : lu_lead(n) + (s - 1) * kOuter;
  return k < n ? k : n;
}
// width of the step that starts at column K0
__host__ __device__ __forceinline__ int lu_kb(int n, int K0) {
  const int w = K0 == 0 ? lu_lead(n) : kOuter;
  const int kb = w < n - K0 ? w : n - K0;
  __builtin_assume(kb <= kOuter);
  return kb;
}
// index of the step that starts at column K0
__host__ __device__ __forceinline__ int lu_step(int n, int K0) { return K0 == 0 ? 0 : (K0 - lu_lead(n)) / kOuter + 1; }

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));

// Matrix data is reached through pointers held in the work lists; they are
// declared in the global address space so that the compiler emits global
// (not flat) memory instructions: a flat load also counts against the LDS
// wait counter, so every LDS wait would wait for the global prefetches too.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) int32_t gint;

struct GemmLds {
  double Lt[kGK][kGT + kPad];   // -A[r, k] chunk, transposed
  double Ut[kGK][kGT + kPad];   //  A[k, c] chunk
};

// One output tile of the product below: rows [rt, min(r1, rt + RT)), columns
// [ct, min(c1, ct + CT)) with RT = WR 16 BI and CT = (NW / WR) 16 BJ -- WR x
// (NW / WR) wavefronts of 16 BI x 16 BJ outputs each.  The operand chunks are
// staged in LDS at the full 128 x 128 tile's shape either way (entries beyond
// the tile are zero); the shape only sets how many MFMAs each wavefront runs.
template <bool SET, int NT, int WR, int BI, int BJ>
__device__ __attribute__((always_inline)) void gemm_tile(gdouble* __restrict__ A, int ld, int rt, int r1, int ct,
                                                          int c1, int k0, int k1, const gdouble* Lb, int ldl,
                                                          int lro, int lko, GemmLds& s) {
  constexpr int NW = NT / kWave, WC = NW / WR;
  constexpr int RW = 16 * BI, CW = 16 * BJ;          // outputs per wavefront
  static_assert(WR * RW <= kGT && WC * CW <= kGT && WR * WC == NW, "tile shape");
  // K chunk: 32 with 512 threads; 16 with 256, whose 64 x 64 accumulators
  // leave registers for half as many prefetched operands
  constexpr int KC = NT >= 512 ? kGK : kGK / 2;
  constexpr int LP = NT / KC, LIT = kGT / LP;        // A[r, k] chunk: rows per pass, passes
  constexpr int UP = NT / kGT, UIT = KC / UP;        // A[k, c] chunk
  static_assert(BI * 4 <= 32 && LIT <= 32, "mask widths");
  // element offsets from A fit in 32 bits (n * ld < 2^31)
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w / WC, wc = w % WC;
  const int li = lane & 15, lk = lane >> 4;
  const int lrow = tid / KC, lcol = tid % KC;        // operand loads: A[r, k] chunk
  const int urow = tid / kGT, ucol = tid % kGT;      //                A[k, c] chunk
  double* __restrict__ lt_st = &s.Lt[lcol][lrow];
  double* __restrict__ ut_st = &s.Ut[urow][ucol];
  const double* __restrict__ lt_rd = &s.Lt[lk][RW * wr + li];
  const double* __restrict__ ut_rd = &s.Ut[lk][CW * wc + li];
  const int crow = rt + RW * wr + lk, ccol = ct + CW * wc + li;
  const int coff = crow * ld + ccol;
  unsigned rmask = 0, cmask = 0;
#pragma unroll
  for (int t = 0; t < 4 * BI; ++t)   // t = 4 bi + v: row offset 16 bi + 4 v
    rmask |= (crow + 16 * (t >> 2) + 4 * (t & 3) < r1) ? (1u << t) : 0u;
#pragma unroll
  for (int bj = 0; bj < BJ; ++bj) cmask |= (ccol + 16 * bj < c1) ? (1u << bj) : 0u;
  // the product accumulates from zero; the tile itself is read only at
  // the end, a block row at a time (few registers in flight)
  dbl4 acc[BI][BJ];
#pragma unroll
  for (int bi = 0; bi < BI; ++bi)
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) acc[bi][bj] = dbl4{0.0, 0.0, 0.0, 0.0};
  const int loff = (rt - lro + lrow) * ldl + lcol - lko;
  const int uoff = urow * ld + ct + ucol;
  unsigned lmask = 0;
#pragma unroll
  for (int it = 0; it < LIT; ++it) lmask |= (rt + lrow + LP * it < r1) ? (1u << it) : 0u;
  const bool ucol_ok = ct + ucol < c1;
  double pl[LIT], pu[UIT];
  // fetch issues the chunk's loads (raw values: out-of-range entries read
  // the valid A[0]); stage zeroes those entries on their way into LDS --
  // masking at the load would make the wavefront wait for the prefetch
  // before the products that were to hide it
  auto fetch = [&](int kc) {
    const bool lk_ok = kc + lcol < k1;
#pragma unroll
    for (int it = 0; it < LIT; ++it) {
      const bool okl = lk_ok && ((lmask >> it) & 1u);
      pl[it] = Lb[okl ? loff + LP * it * ldl + kc : 0];
    }
#pragma unroll
    for (int it = 0; it < UIT; ++it) {
      const bool oku = ucol_ok && kc + urow + UP * it < k1;
      pu[it] = A[oku ? uoff + (kc + UP * it) * ld : 0];
    }
  };
  auto stage = [&](int off, int kc) {  // the chunk fetched at kc into LDS rows [off, off + KC)
    const bool lk_ok = kc + lcol < k1;
#pragma unroll
    for (int it = 0; it < LIT; ++it) {
      const bool okl = lk_ok && ((lmask >> it) & 1u);
      lt_st[off * (kGT + kPad) + LP * it] = okl ? (SET ? pl[it] : -pl[it]) : 0.0;
    }
#pragma unroll
    for (int it = 0; it < UIT; ++it) {
      const bool oku = ucol_ok && kc + urow + UP * it < k1;
      ut_st[off * (kGT + kPad) + UP * it * (kGT + kPad)] = oku ? pu[it] : 0.0;
    }
  };
  auto products = [&](int off) {       // the MFMAs of the chunk in LDS rows [off, off + KC)
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      double a[BI], b[BJ];
#pragma unroll
      for (int bi = 0; bi < BI; ++bi) a[bi] = lt_rd[(off + 4 * ks) * (kGT + kPad) + 16 * bi];
#pragma unroll
      for (int bj = 0; bj < BJ; ++bj) b[bj] = ut_rd[(off + 4 * ks) * (kGT + kPad) + 16 * bj];
#pragma unroll
      for (int bi = 0; bi < BI; ++bi)
#pragma unroll
        for (int bj = 0; bj < BJ; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
    }
  };
  fetch(k0);
  if (2 * KC <= kGK) {
    // two LDS buffers (rows [0, KC) and [KC, 2 KC)): the next chunk is
    // staged while the other wavefronts may still read the current one,
    // one barrier per chunk
    stage(0, k0);
    __syncthreads();
    int cur = 0;
#pragma unroll 1
    for (int kc = k0; kc < k1; kc += KC) {
      const bool more = kc + KC < k1;
      if (more) fetch(kc + KC);
      products(cur);
      if (more) stage(KC - cur, kc + KC);
      __syncthreads();
      cur = KC - cur;
    }
  } else {
#pragma unroll 1
    for (int kc = k0; kc < k1; kc += KC) {
      stage(0, kc);
      __syncthreads();
      if (kc + KC < k1) fetch(kc + KC);
      products(0);
      __syncthreads();
    }
  }
#pragma unroll
  for (int bi = 0; bi < BI; ++bi) {
    double cv[4][BJ];
    if (!SET) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int bj = 0; bj < BJ; ++bj) {
          const bool ok = ((rmask >> (4 * bi + v)) & (cmask >> bj) & 1u) != 0;
          cv[v][bj] = A[ok ? coff + (16 * bi + 4 * v) * ld + 16 * bj : 0];
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int bj = 0; bj < BJ; ++bj) {
        const bool ok = ((rmask >> (4 * bi + v)) & (cmask >> bj) & 1u) != 0;
        if (ok) A[coff + (16 * bi + 4 * v) * ld + 16 * bj] = SET ? acc[bi][bj][v] : cv[v][bj] + acc[bi][bj][v];
      }
  }
}

// A[r0:r1, c0:c1] -= A[r0:r1, k0:k1] A[k0:k1, c0:c1]; the three blocks are
// disjoint.  Called by all NT threads of the workgroup; ends with a barrier.
// NT = 512: 4 x 2 wavefronts of 32 x 64 outputs; NT = 256: 2 x 2 wavefronts
// of 64 x 64 (twice the MFMAs per LDS operand read, and two workgroups share
// a CU, so that one's tile loads and stores overlap the other's products).
// With 256 threads a block of one tile that ends inside the 128 x 128 grid
// takes a smaller shape, picked once (no branch inside the K loop): 64 rows
// (2 x 2 wavefronts of 32 x 64), 64 columns (of 64 x 32), both (32 x 32),
// or 80 columns -- the 65 right-hand sides padded to 80 -- as 4 x 1
// wavefronts of 32 x 80 (16 x 80 with 64 rows).  Without them every step's
// last row tile and last column tile cost a full tile of MFMAs.
// Addresses are one per-lane base pointer plus workgroup-uniform offsets, and
// the edge tests are per-lane bit masks, to keep register use low.
// SET: A[r0:r1, c0:c1] = Lb[r - lro, k - lko] A[k0:k1, c0:c1] with a separate
// left factor Lb (leading dimension ldl); the right factor may be the output
// block itself (every read precedes the final barrier, every write follows it).
template <bool SET, int NT>
__device__ __attribute__((always_inline)) void gemm_op(gdouble* __restrict__ A, int ld, int r0, int r1, int c0, int c1,
                                                        int k0, int k1, const gdouble* Lb, int ldl, int lro, int lko,
                                                        GemmLds& s) {
  if constexpr (NT == 256) {
    if (r1 - r0 <= kGT && c1 - c0 <= kGT) {   // one tile (every LU launch's unit): pick its shape
      const bool short_r = r1 - r0 <= kGT / 2;
      const int wcols = c1 - c0;
      if (wcols > 80) {
        if (short_r) gemm_tile<SET, NT, 2, 2, 4>(A, ld, r0, r1, c0, c1, k0, k1, Lb, ldl, lro, lko, s);
        else gemm_tile<SET, NT, 2, 4, 4>(A, ld, r0, r1, c0, c1, k0, k1, Lb, ldl, lro, lko, s);
      } else if (wcols > 64) {
        if (short_r) gemm_tile<SET, NT, 4, 1, 5>(A, ld, r0, r1, c0, c1, k0, k1, Lb, ldl, lro, lko, s);
        else gemm_tile<SET, NT, 4, 2, 5>(A, ld, r0, r1, c0, c1, k0, k1, Lb, ldl, lro, lko, s);
      } else {
        if (short_r) gemm_tile<SET, NT, 2, 2, 2>(A, ld, r0, r1, c0, c1, k0, k1, Lb, ldl, lro, lko, s);
        else gemm_tile<SET, NT, 2, 4, 2>(A, ld, r0, r1, c0, c1, k0, k1, Lb, ldl, lro, lko, s);
      }
      __syncthreads();
      return;
    }
  }
  constexpr int WR = NT == 512 ? 4 : 2, BI = NT == 512 ? 2 : 4;
#pragma unroll 1
  for (int rt = r0; rt < r1; rt += kGT) {
#pragma unroll 1
    for (int ct = c0; ct < c1; ct += kGT) gemm_tile<SET, NT, WR, BI, 4>(A, ld, rt, r1, ct, c1, k0, k1, Lb, ldl, lro, lko, s);
  }
  __syncthreads();
}

template <int NT>
__device__ __attribute__((always_inline)) void gemm_sub(gdouble* __restrict__ A, int ld, int r0, int r1, int c0, int c1,
                                                         int k0, int k1, GemmLds& s) {
  gemm_op<false, NT>(A, ld, r0, r1, c0, c1, k0, k1, A, ld, 0, 0, s);
}

// Narrow update A[r0:r1, c0:c1] -= A[r0:r1, k0:k1] A[k0:k1, c0:c1] for
// k1 - k0 <= 32 and c1 - c0 <= 128 (the updates inside a panel or a 128-row
// block): the small right factor is staged in LDS once, then every wavefront
// streams its own 16-row strips -- left factor in the MFMA A layout and the
// strip of C loaded straight from global memory, no barrier between strips.
// Ends with a barrier.
__device__ __attribute__((always_inline)) void strip_update(gdouble* __restrict__ A, int ld, int r0, int r1,
                                                             int c0, int c1, int k0, int k1,
                                                             double (*sU)[kGT + kPad]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int K = k1 - k0, W = c1 - c0;
#pragma unroll 1
  for (int idx = tid; idx < kGK * kGT; idx += kThreads) {
    const int k = idx / kGT, c = idx - k * kGT;
    sU[k][c] = (k < K && c < W) ? A[(k0 + k) * ld + c0 + c] : 0.0;
  }
  __syncthreads();
  const int KS = (K + 3) >> 2, CB = (W + 15) >> 4;
  const int nstrips = (r1 - r0 + 15) >> 4;
#pragma unroll 1
  for (int sidx = w; sidx < nstrips; sidx += kThreads / kWave) {
    const int rs = r0 + 16 * sidx;
    double a[kGK / 4];
#pragma unroll
    for (int ks = 0; ks < kGK / 4; ++ks) {
      const bool ok = ks < KS && rs + li < r1 && 4 * ks + lk < K;
      const double v = A[ok ? (rs + li) * ld + k0 + 4 * ks + lk : 0];
      a[ks] = ok ? -v : 0.0;
    }
    // two 16-column blocks at a time (keeps the live registers low)
#pragma unroll 1
    for (int cq = 0; cq < CB; cq += 2) {
      dbl4 acc[2];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int cb = cq + u;
          const bool ok = cb < CB && rs + 4 * v + lk < r1 && 16 * cb + li < W;
          const double x = A[ok ? (rs + 4 * v + lk) * ld + c0 + 16 * cb + li : 0];
          acc[u][v] = ok ? x : 0.0;
        }
#pragma unroll
      for (int ks = 0; ks < kGK / 4; ++ks) {
        if (ks < KS) {
#pragma unroll
          for (int u = 0; u < 2; ++u)
            if (cq + u < CB)
              acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], sU[4 * ks + lk][16 * (cq + u) + li], acc[u], 0, 0, 0);
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int cb = cq + u;
          if (cb < CB && rs + 4 * v + lk < r1 && 16 * cb + li < W)
            A[(rs + 4 * v + lk) * ld + c0 + 16 * cb + li] = acc[u][v];
        }
    }
  }
  __syncthreads();
}

// Triangular blocks (w <= NB <= 32 rows) are solved through their explicit
// inverse: one wavefront inverts the w x w diagonal block column by column
// (lane j forms column j with fully unrolled substitution), then every
// wavefront multiplies 16-column blocks of the right-hand side by it on MFMA.
struct TriLds {
  double blk[32][33];   // the diagonal block, zero-padded
  double inv[32][33];   // its inverse, zero-padded
  double inv2[32][33];  // tri_inverse_pair: the inverse of its upper triangle
};

// T = (unit lower triangle of A[a:a+w, a:a+w])^-1 if LOWER, else
// (upper triangle with diagonal)^-1.  Ends with a barrier.
template <int NB, bool LOWER>
__device__ __attribute__((always_inline)) void tri_inverse(const gdouble* __restrict__ A, int ld, int a,
                                                            int w, TriLds& t) {
  const int tid = threadIdx.x;
  for (int idx = tid; idx < NB * NB; idx += kThreads) {
    const int i = idx / NB, j = idx - i * NB;
    t.blk[i][j] = (i < w && j < w) ? A[(a + i) * ld + a + j] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  if (tid < NB) {
    // lane j forms column j of the inverse in place in t.inv (its own column
    // only, so no synchronisation is needed inside the substitution)
    const int j = tid;
    if (LOWER) {
#pragma unroll 1
      for (int i = 0; i < NB; ++i) {
        double v = (i == j) ? 1.0 : 0.0;
#pragma unroll 8
        for (int k = 0; k < i; ++k) v -= t.blk[i][k] * t.inv[k][j];
        t.inv[i][j] = v;
      }
    } else {
#pragma unroll 1
      for (int i = NB - 1; i >= 0; --i) {
        double v = (i == j) ? 1.0 : 0.0;
#pragma unroll 8
        for (int k = i + 1; k < NB; ++k) v -= t.blk[i][k] * t.inv[k][j];
        t.inv[i][j] = v / t.blk[i][i];
      }
    }
#pragma unroll 1
    for (int i = 0; i < NB; ++i)
      if (i >= w || j >= w) t.inv[i][j] = 0.0;
  }
  __syncthreads();
}

// Both inverses of one kTB x kTB diagonal block: t.inv <- (unit lower)^-1 by
// wavefront 0 and t.inv2 <- (upper with diagonal)^-1 by wavefront 1, at the
// same time.  Ends with a barrier.
__device__ __attribute__((always_inline)) void tri_inverse_pair(const gdouble* __restrict__ A, int ld, int a,
                                                                 int w, TriLds& t) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int idx = tid; idx < kTB * kTB; idx += kThreads) {
    const int i = idx / kTB, j = idx - i * kTB;
    t.blk[i][j] = (i < w && j < w) ? A[(a + i) * ld + a + j] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  if (wv == 0 && lane < kTB) {
    const int j = lane;
#pragma unroll 1
    for (int i = 0; i < kTB; ++i) {
      double v = (i == j) ? 1.0 : 0.0;
#pragma unroll 8
      for (int k = 0; k < i; ++k) v -= t.blk[i][k] * t.inv[k][j];
      t.inv[i][j] = v;
    }
#pragma unroll 1
    for (int i = 0; i < kTB; ++i)
      if (i >= w || j >= w) t.inv[i][j] = 0.0;
  } else if (wv == 1 && lane < kTB) {
    const int j = lane;
#pragma unroll 1
    for (int i = kTB - 1; i >= 0; --i) {
      double v = (i == j) ? 1.0 : 0.0;
#pragma unroll 8
      for (int k = i + 1; k < kTB; ++k) v -= t.blk[i][k] * t.inv2[k][j];
      t.inv2[i][j] = v / t.blk[i][i];
    }
#pragma unroll 1
    for (int i = 0; i < kTB; ++i)
      if (i >= w || j >= w) t.inv2[i][j] = 0.0;
  }
  __syncthreads();
}

// Rows [a, a+w) of columns [c0, c1) <- T (rows), T = t.inv (w <= NB).  Each
// wavefront takes 16-column blocks; the block's w rows are loaded in the MFMA
// B layout, multiplied by T read from LDS as the products need it (few live
// registers), and written back in place.  Ends with a barrier.
template <int NB>
__device__ __attribute__((always_inline)) void tri_apply(gdouble* __restrict__ A, int ld, int a, int w,
                                                          int c0, int c1, const TriLds& t) {
  constexpr int BI = NB / 16, KS = NB / 4;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int roff = (a + lk) * ld;
#pragma unroll 1
  for (int cb = c0 + 16 * wv; cb < c1; cb += 16 * (kThreads / kWave)) {
    const int col = cb + li;
    const bool cok = col < c1;
    double xb[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const bool ok = cok && 4 * ks + lk < w;
      const double v = A[ok ? roff + 4 * ks * ld + col : 0];
      xb[ks] = ok ? v : 0.0;
    }
    dbl4 acc[BI];
#pragma unroll
    for (int bi = 0; bi < BI; ++bi) acc[bi] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int bi = 0; bi < BI; ++bi)
        acc[bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(t.inv[16 * bi + li][4 * ks + lk], xb[ks], acc[bi], 0, 0, 0);
#pragma unroll
    for (int bi = 0; bi < BI; ++bi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * bi + 4 * v + lk;
        if (cok && r < w) A[(a + r) * ld + col] = acc[bi][v];
      }
  }
  __syncthreads();
}

}  // namespace

// Per-matrix work area of one step (global memory).
// The records read by the U-row tiles are kept for two steps (index: step
// parity), since the tiles of step s run beside the panel of step s + 1.
struct LuWork {
  double linv[2][kOuter][kOuter];      // L11^-1 (unit lower), zero-padded
  double inv[kOuter / kTB][kTB][kTB];  // inverses of L11's unit-lower diagonal blocks
  int rows[2][2 * kOuter];             // rows touched by the step's interchanges
  int src[2][2 * kOuter];              // slot whose old contents end up in each slot's row
  int count[2];
  int pad[62];
};
static_assert(sizeof(LuWork) % 8 == 0, "the inverses of U's blocks follow LuWork");

typedef __attribute__((address_space(1))) LuWork gwork;

// A work-list entry as the kernels see it (global address space pointers).
struct GItem {
  gdouble* A;
  gint* piv;
  gint* status;
  gwork* work;
  gdouble* uinv;
  int32_t n, ld, nrhs, cls;
};

__device__ __forceinline__ GItem gitem(const LuItem& it) {
  return GItem{(gdouble*)it.A, (gint*)it.piv, (gint*)it.status, (gwork*)it.work, (gdouble*)it.uinv,
               it.n, it.ld, it.nrhs, it.cls};
}

namespace {

// Composes the interchanges (base + t) <-> piv[t], t = 0..cnt-1 in order
// (cnt <= 128), into one permutation of at most 2 cnt rows: rows[e] receives
// the old contents of rows[src[e]].  slot[r] locates row r among the rows
// added below the block (-1: not yet added); it must be -1 for every row on
// entry and is restored on return, so each interchange costs O(1).  Run by
// one thread on LDS arrays.
__device__ void compose_perm(const int* __restrict__ piv, int base, int cnt, int* __restrict__ rows,
                             int* __restrict__ src, int* __restrict__ count, short* __restrict__ slot) {
  int nt = cnt;
  for (int t = 0; t < cnt; ++t) {
    rows[t] = base + t;
    src[t] = t;
  }
  for (int t = 0; t < cnt; ++t) {
    const int b = piv[t];
    if (b == base + t) continue;
    int sb;
    if (b < base + cnt) {
      sb = b - base;
    } else {
      sb = slot[b];
      if (sb < 0) {
        sb = nt++;
        rows[sb] = b;
        src[sb] = sb;
        slot[b] = (short)sb;
      }
    }
    const int tmp = src[t];
    src[t] = src[sb];
    src[sb] = tmp;
  }
  for (int e = cnt; e < nt; ++e) slot[rows[e]] = -1;
  *count = nt;
}

struct PermLds {
  int rows[2 * kOuter];
  int src[2 * kOuter];
  int count;
};

// Applies a composed permutation to columns [lo, hi) except [skip0, skip1):
// row rows[e] receives the old contents of row rows[src[e]].  In chunks of
// columns whose moved entries fit in registers (32 per thread): every read
// of a chunk precedes every write of it (one barrier), no LDS staging, and
// the next chunk's reads (other columns) follow the writes at once.  Ends
// with a barrier.
template <int NT>
__device__ __attribute__((always_inline)) void apply_perm(gdouble* __restrict__ A, int ld, const PermLds& pl,
                                                           int lo, int hi, int skip0, int skip1) {
  constexpr int CH = NT >= 512 ? 64 : 32;          // columns per chunk
  constexpr int V = 2 * kOuter * CH / NT;          // entries per thread
  const int tid = threadIdx.x;
  const int nt = pl.count;
  for (int c0 = lo; c0 < hi; c0 += CH) {
    double val[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const int idx = tid + NT * k, e = idx / CH, c = c0 + idx % CH;
      const bool ok = e < nt && c < hi && !(c >= skip0 && c < skip1);
      val[k] = A[ok ? pl.rows[pl.src[ok ? e : 0]] * ld + c : 0];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const int idx = tid + NT * k, e = idx / CH, c = c0 + idx % CH;
      const bool ok = e < nt && c < hi && !(c >= skip0 && c < skip1);
      if (ok) A[pl.rows[e] * ld + c] = val[k];
    }
  }
  __syncthreads();
}

// Wavefront maximum of a double: DPP exchanges inside each row of 16 lanes
// (quad permutations, half-row and row mirrors), then the four row maxima
// read from lanes 0, 16, 32, 48.  fmax drops NaN operands.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Wavefront maximum of a 32-bit unsigned value, in every lane: DPP maxima
// inside each row of 16 lanes, then row_bcast15 / row_bcast31 carry the row
// maxima into lane 63.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xb1, 0xf, 0xf, false));   // quad_perm [1,0,3,2]
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4e, 0xf, 0xf, false));   // quad_perm [2,3,0,1]
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false));  // row_half_mirror
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false));  // row_mirror
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast15
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast31
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Wavefront maximum of a 64-bit unsigned value: the high words, then the low
// words of the lanes whose high word is the maximum.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  const unsigned hi = (unsigned)(v >> 32), lo = (unsigned)v;
  const unsigned mh = wave_max_u32(hi);
  const unsigned ml = wave_max_u32(hi == mh ? lo : 0u);
  return ((unsigned long long)mh << 32) | ml;
}

__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_f64<0xb1>(v));    // quad_perm [1, 0, 3, 2]
  v = fmax(v, dpp_f64<0x4e>(v));    // quad_perm [2, 3, 0, 1]
  v = fmax(v, dpp_f64<0x141>(v));   // row_half_mirror
  v = fmax(v, dpp_f64<0x140>(v));   // row_mirror
  return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)), fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// LDS of the sub-panel factorisation: per column, each wavefront's best pivot
// candidate (value, row index, full sub-panel row) and the current row kk,
// double-buffered by column parity so that one barrier per column suffices.
template <int NB>
struct PanelLds {
  double cand[2][kThreads / kWave][NB];
  double krow[2][NB];
  double cv[2][kThreads / kWave];
  int ci[2][kThreads / kWave];
};

// Factorises the sub-panel A[k0:n, k0:k0+pw] (pw <= NB) held in registers:
// thread t owns rows k0 + t + kThreads s.  The column index is a compile-time
// constant in the unrolled loop, so the register file is never indexed
// dynamically.  Pivot: largest magnitude, lowest row index on ties.
template <int ROWS, int NB>
__device__ __attribute__((always_inline)) void factor_subpanel(gdouble* __restrict__ A, int ld, int n,
                                                                int k0, int pw, int K0,
                                                                int* __restrict__ s_piv,
                                                                gint* __restrict__ piv,
                                                                PanelLds<NB>& pl, int& singular) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double P[ROWS][NB];
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int row = k0 + tid + kThreads * s;
#pragma unroll
    for (int c = 0; c < NB; ++c) P[s][c] = (row < n && c < pw) ? A[row * ld + k0 + c] : 0.0;
  }
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c < pw) {                            // uniform
      const int kk = k0 + c, buf = c & 1;
      // the wavefront's largest magnitude (NaN never wins), then the lowest
      // of its rows holding it: both wavefront-uniform
      double lv = -1.0;
#pragma unroll
      for (int s = 0; s < ROWS; ++s) {
        const int row = k0 + tid + kThreads * s;
        if (row >= kk && row < n) lv = fmax(lv, fabs(P[s][c]));
      }
      const double wmax = wave_max(lv);
      double bv = -1.0;
      int bi = 0x7fffffff;
#pragma unroll
      for (int s = 0; s < ROWS; ++s) {
        const int row = k0 + tid + kThreads * s;
        const unsigned long long m = __ballot(row >= kk && row < n && fabs(P[s][c]) == wmax);
        if (bi == 0x7fffffff && m != 0ull) {
          bi = k0 + kWave * w + __builtin_ctzll(m) + kThreads * s;
          bv = wmax;
        }
      }
#pragma unroll
      for (int s = 0; s < ROWS; ++s) {
        const int row = k0 + tid + kThreads * s;
        if (row == bi)
#pragma unroll
          for (int cc = 0; cc < NB; ++cc) pl.cand[buf][w][cc] = P[s][cc];
      }
      if (lane == 0) { pl.cv[buf][w] = bv; pl.ci[buf][w] = bi; }
      if (tid == c)
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) pl.krow[buf][cc] = P[0][cc];
      __syncthreads();
      double gv = pl.cv[buf][0];
      int gi = pl.ci[buf][0], gw = 0;
#pragma unroll
      for (int t = 1; t < kThreads / kWave; ++t) {
        const double ov = pl.cv[buf][t];
        const int oi = pl.ci[buf][t];
        if (ov > gv || (ov == gv && oi < gi)) { gv = ov; gi = oi; gw = t; }
      }
      const bool ok = gv > 0.0;
      if (!ok) singular = 1;
      const int p = ok ? gi : kk;
      const double* prow = ok ? pl.cand[buf][gw] : pl.krow[buf];
      if (p != kk) {
#pragma unroll
        for (int s = 0; s < ROWS; ++s) {
          const int row = k0 + tid + kThreads * s;
          if (row == p)
#pragma unroll
            for (int cc = 0; cc < NB; ++cc) P[s][cc] = pl.krow[buf][cc];
        }
      }
      if (tid == c)
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) P[0][cc] = prow[cc];
      if (ok) {
        const double inv = 1.0 / prow[c];
#pragma unroll
        for (int s = 0; s < ROWS; ++s) {
          const int row = k0 + tid + kThreads * s;
          if (row > kk && row < n) {
            const double l = P[s][c] * inv;
            P[s][c] = l;
#pragma unroll
            for (int cc = 0; cc < NB; ++cc)
              if (cc > c) P[s][cc] -= l * prow[cc];
          }
        }
      }
      if (tid == 0) {
        s_piv[kk - K0] = p;
        piv[kk] = p;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int row = k0 + tid + kThreads * s;
    if (row < n)
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < pw) A[row * ld + k0 + c] = P[s][c];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Work bodies.  Each acts on one matrix (or one tile of it); the scheduled
// kernels below pick the matrix and tile from a work list.

union MatLds {
  GemmLds g;
  TriLds t;
};

// The panel kernel's LDS (about 38 KB, so that LDS never limits it below
// the two workgroups per CU its registers allow).
union PanelScratch {
  double sU[kGK][kGT + kPad];   // strip_update's right factor, apply_perm's staging
  TriLds t;
};

constexpr int kMaxOrder = 4096;   // largest matrix order of the panel classes

template <int NB>
struct PanelShared {
  PanelScratch u;
  PanelLds<NB> pl;
  int piv[kOuter];
  PermLds perm;
  short slot[kMaxOrder];        // compose_perm's row -> slot map
};

template <int ROWS, int NB>
__device__ __attribute__((always_inline)) void panel_body(const GItem& it, int K0, PanelShared<NB>& sh) {
  constexpr int TB = NB < 16 ? 16 : NB;
  gdouble* A = it.A;
  const int n = it.n, ld = it.ld;
  gwork* W = it.work;
  const int tid = threadIdx.x;
  const int kb = lu_kb(n, K0);
  int singular = 0;
  for (int r = tid; r < n; r += kThreads) sh.slot[r] = -1;
  // groups of kTB columns, each factorised by sub-panels of NB columns; the
  // group's update of the rest of the panel uses K = kTB
  for (int b = 0, g0 = K0; g0 < K0 + kb; ++b, g0 += kTB) {
    const int gw = min(kTB, K0 + kb - g0);
    for (int k0 = g0; k0 < g0 + gw; k0 += NB) {
      const int pw = min(NB, g0 + gw - k0);
      factor_subpanel<ROWS, NB>(A, ld, n, k0, pw, K0, sh.piv, it.piv, sh.pl, singular);
      if (tid == 0)
        compose_perm(sh.piv + (k0 - K0), k0, pw, sh.perm.rows, sh.perm.src, &sh.perm.count, sh.slot);
      __syncthreads();
      // the sub-panel's interchanges on the rest of the panel
      apply_perm<kThreads>(A, ld, sh.perm, K0, K0 + kb, k0, k0 + pw);
      if (k0 + pw < g0 + gw) {
        tri_inverse<TB, true>(A, ld, k0, pw, sh.u.t);
        tri_apply<TB>(A, ld, k0, pw, k0 + pw, g0 + gw, sh.u.t);
        strip_update(A, ld, k0 + pw, n, k0 + pw, g0 + gw, k0, k0 + pw, sh.u.sU);
      }
    }
    // the group's diagonal block is final: keep the inverse of its upper
    // triangle for the back substitution and that of its unit-lower triangle
    // for the U12 tiles
    tri_inverse_pair(A, ld, g0, gw, sh.u.t);
    for (int idx = tid; idx < kTB * kTB; idx += kThreads) {
      it.uinv[(g0 / kTB) * kTB * kTB + idx] = sh.u.t.inv2[idx >> 5][idx & 31];
      W->inv[b][idx >> 5][idx & 31] = sh.u.t.inv[idx >> 5][idx & 31];
    }
    if (g0 + gw < K0 + kb) {
      tri_apply<kTB>(A, ld, g0, gw, g0 + gw, K0 + kb, sh.u.t);
      strip_update(A, ld, g0 + gw, n, g0 + gw, K0 + kb, g0, g0 + gw, sh.u.sU);
    }
    __syncthreads();
  }
  const int par = lu_step(n, K0) & 1;
  // the step's composed permutation, formed in LDS and copied out
  if (tid == 0) compose_perm(sh.piv, K0, kb, sh.perm.rows, sh.perm.src, &sh.perm.count, sh.slot);
  __syncthreads();
  const int nt = sh.perm.count;
  for (int e = tid; e < nt; e += kThreads) {
    W->rows[par][e] = sh.perm.rows[e];
    W->src[par][e] = sh.perm.src[e];
  }
  if (tid == 0) W->count[par] = nt;
  if (tid == 0 && (K0 == 0 || singular)) *it.status = singular;
}

// ---------------------------------------------------------------------------
// Panel with row ownership (panel heights up to kOwnMax).  Thread t keeps
// physical row K0 + t of the panel for the whole step and tracks that row's
// position in the pivoted order; rows are not interchanged while the panel
// is factorised.  The pivot of column K0 + c is the largest magnitude among
// the rows at positions >= c (the lowest position on ties) -- the row that
// partial pivoting with interchanges picks -- and every row sees the same
// operations in the same order, so the factors are those of the interchange
// form.  Columns are taken in groups of kTB: a group is factorised in
// registers (one barrier per column), its diagonal block is inverted in LDS,
// its pivot rows of the trailing panel columns become U12 = L11^-1 A12 and
// the remaining rows take the rank-kTB update on MFMA.  At the end the rows
// that moved are written to their positions once, and the step's composed
// permutation is recorded for the other columns.

constexpr int kOwnMax = 1024;
constexpr int kSW = kOuter - kTB;            // trailing panel columns of a group (at most)

// The phases of a group use the LDS in turn (about 27 KB in all, so that
// up to five workgroups share a CU).
struct OwnLds {
  union {
    struct {                                   // column factorisation
      double cand[2][kOwnMax / kWave][kTB];   // each wavefront's best candidate row
      unsigned long long ckey[2][kOwnMax / kWave];
      int cpos[2][kOwnMax / kWave];
      int crow[2][kOwnMax / kWave];
    } f;
    TriLds t;                                  // the group's diagonal block and its inverses
    double S[kTB][kSW + kPad];                 // U12: the group's pivot rows of the trailing columns
    struct {                                   // the step's permutation record
      short who[kOwnMax];                      // the physical row (- K0) at each position
      short slot[kOwnMax];                     // moved rows: index in the record
      int wcount[kOwnMax / kWave];
    } g;
  } u;
  short pos[kOwnMax];                          // position of physical row K0 + t
  int prow[kTB];                               // physical rows (- K0) of the group's pivots
};

typedef __attribute__((address_space(3))) double ldouble;

// An LDS address the compiler treats as opaque: a per-lane choice between
// two LDS arrays would otherwise be folded into every access as a pair of
// constants (one register each).
__device__ __forceinline__ ldouble* opaque_lds(ldouble* p) {
  uint32_t a = (uint32_t)(size_t)p;
  __asm__ volatile("" : "+v"(a));
  return (ldouble*)(size_t)a;
}

// Step K of the register-resident triangular inverse (below).  Empty asm
// statements pin the order: every x_i of step K passes through one after its
// product, and the base address of B through one after them, so the loads
// of step K + 1 are issued only after the products of step K (left alone,
// the compiler issues all loads at once and spills their results).
template <int K>
__device__ __attribute__((always_inline)) void inv_step(double (&x)[kTB], const ldouble*& bb, bool lo) {
  constexpr int R = kTB + 1;
  // (division by one, exact, in the lower half: no branch)
  x[K] = x[K] / (lo ? 1.0 : bb[R * K + K]);
  // chunks of 8 products, each chunk's loads issued after the previous
  // chunk's products
#pragma unroll
  for (int i0 = K + 1; i0 < kTB; i0 += 8) {
    const ldouble* __restrict__ b = bb;
#pragma unroll
    for (int i = i0; i < i0 + 8 && i < kTB; ++i) x[i] -= b[R * i + K] * x[K];
#pragma unroll
    for (int i = i0; i < i0 + 8 && i < kTB; ++i) __asm__ volatile("" : "+v"(x[i]));
    uint32_t a = (uint32_t)(size_t)bb;
    __asm__ volatile("" : "+v"(a));
    bb = (const ldouble*)(size_t)a;
  }
}

template <int... Ks>
__device__ __attribute__((always_inline)) void inv_steps(std::integer_sequence<int, Ks...>, double (&x)[kTB],
                                                          const ldouble* bb, bool lo) {
  (inv_step<Ks>(x, bb, lo), ...);
}

// Both inverses of the kTB x kTB block in t.blk (identity-padded beyond w,
// and held reversed, t.inv2[i][k] = t.blk[31 - i][31 - k], on entry):
// t.inv <- (unit lower)^-1, t.inv2 <- (upper with diagonal)^-1, by
// wavefront 0: lane j < 32 forms column j of the lower inverse from t.blk,
// lane 32 + j column j of the upper one in reversed index order from the
// reversed copy, so that both run the same forward substitution with the
// same LDS offsets (the upper result overwrites the copy after every read
// of it: one wavefront runs in order).  The column is held in registers
// and updated right-looking -- x_i -= B(i, k) x_k for every i > k as soon as
// x_k is final -- which subtracts the same terms in the same order as the
// row-by-row form, so the result is identical while the chain between
// successive x_k is one product.  Ends with a barrier.
__device__ __attribute__((always_inline)) void own_block_inverses(int w, TriLds& t) {
  const int tid = threadIdx.x;
  if (tid < 2 * kTB) {
    constexpr int R = kTB + 1;               // row stride of the LDS blocks
    const bool lo = tid < kTB;
    const int j = tid & (kTB - 1);
    const int sg = lo ? 1 : -1;
    // B(i, k) = bb[R i + k]: lower blk[i][k], upper blk[31 - i][31 - k]
    const ldouble* __restrict__ bb = opaque_lds(lo ? (ldouble*)&t.blk[0][0] : (ldouble*)&t.inv2[0][0]);
    int target = lo ? j : kTB - 1 - j;
    __asm__ volatile("" : "+v"(target));     // (or the start columns are hoisted out of the group loop and spilled)
    double x[kTB];
#pragma unroll
    for (int i = 0; i < kTB; ++i) x[i] = (i == target) ? 1.0 : 0.0;
    inv_steps(std::make_integer_sequence<int, kTB>{}, x, bb, lo);
    // lower: inv[i][j] = x_i; upper: inv2[31 - i][j] = x_i
    ldouble* xo = opaque_lds(lo ? (ldouble*)&t.inv[0][j] : (ldouble*)&t.inv2[kTB - 1][j]);
#pragma unroll
    for (int i = 0; i < kTB; ++i) xo[sg * R * i] = x[i];
#pragma unroll 1
    for (int i = 0; i < kTB; ++i)
      if (i >= w || j >= w) (lo ? t.inv : t.inv2)[i][j] = 0.0;
  }
  __syncthreads();
}

// Column C of a group (C < gw): pivot search, interchange of positions and
// the rank-1 update of the group's later columns; one barrier.  A template
// per column so that the register row P is only ever indexed by constants.
template <int C>
__device__ __attribute__((always_inline)) void own_column(double (&P)[kTB], int& pos, int& singular, int gw, int g0r,
                                                          int K0, gint* __restrict__ piv, bool own, bool live,
                                                          gdouble* __restrict__ wrow, int nw, OwnLds& sh) {
  if (C >= gw) return;                       // uniform
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int cr = g0r + C, buf = C & 1;
  const bool cand = own && pos >= cr;
  // the candidate's key: the bits of |P[C]|, which order as unsigned
  // integers as the magnitudes do; NaN (never a pivot) and rows that are not
  // candidates have key 0
  const double a = fabs(P[C]);
  const unsigned long long key = (cand && a == a) ? (unsigned long long)__double_as_longlong(a) : 0ull;
  const unsigned long long wkey = wave_max_u64(key);
  const unsigned long long msk = __ballot(cand && key == wkey);
  int wl = -1;
  if (msk != 0ull) {
    wl = __builtin_ctzll(msk);
    if (msk & (msk - 1ull)) {                // ties inside the wavefront: lowest position
      int best = __builtin_amdgcn_readlane(pos, wl);
      for (unsigned long long r = msk & (msk - 1ull); r != 0ull; r &= r - 1ull) {
        const int l = __builtin_ctzll(r);
        const int p = __builtin_amdgcn_readlane(pos, l);
        if (p < best) { best = p; wl = l; }
      }
    }
  }
  if (lane == wl) {
#pragma unroll
    for (int cc = C; cc < kTB; ++cc) sh.u.f.cand[buf][w][cc] = P[cc];
    sh.u.f.ckey[buf][w] = key;
    sh.u.f.cpos[buf][w] = pos;
    sh.u.f.crow[buf][w] = tid;
  }
  if (wl < 0 && lane == 0) {                 // no candidate in this wavefront
    sh.u.f.ckey[buf][w] = 0ull;
    sh.u.f.cpos[buf][w] = 0x7fffffff;
  }
  __syncthreads();
  // the workgroup's pivot: lane v reads wavefront v's record, then the same
  // maximum / lowest-position selection across the lanes
  // (the three records are read at once, in bounds for every lane, and
  // masked afterwards)
  const int vl = lane & (kOwnMax / kWave - 1);
  const unsigned long long okey_raw = sh.u.f.ckey[buf][vl];
  const int opos_raw = sh.u.f.cpos[buf][vl];
  const int orow = sh.u.f.crow[buf][vl];
  const unsigned long long okey = lane < nw ? okey_raw : 0ull;
  const unsigned long long gkey = wave_max_u64(okey);
  const unsigned long long gm = __ballot(lane < nw && okey == gkey);
  int gwv = gm ? __builtin_ctzll(gm) : 0;
  const int opos = lane < nw ? opos_raw : 0x7fffffff;
  int gp = __builtin_amdgcn_readlane(opos, gwv);
  if (gm & (gm - 1ull)) {                    // ties between wavefronts: lowest position
    for (unsigned long long r = gm & (gm - 1ull); r != 0ull; r &= r - 1ull) {
      const int l = __builtin_ctzll(r);
      const int p = __builtin_amdgcn_readlane(opos, l);
      if (p < gp) { gp = p; gwv = l; }
    }
  }
  const bool ok = gkey != 0ull;              // uniform: a nonzero pivot exists
  if (!ok) singular = 1;
  const int ppos = ok ? gp : cr;
  const bool is_piv = ok ? tid == __builtin_amdgcn_readlane(orow, gwv) : (own && pos == cr);
  const int npos = is_piv ? cr : (pos == cr ? ppos : pos);
  if (ok && own && npos > cr) {
    // the pivot row in aligned chunks of 8, each chunk's four 16-byte LDS
    // loads issued together
    const dbl2* __restrict__ pr2 = reinterpret_cast<const dbl2*>(sh.u.f.cand[buf][gwv]);
    double l = 0.0;
#pragma unroll
    for (int q = C / 8; q < kTB / 8; ++q) {
      const dbl2 v0 = pr2[4 * q], v1 = pr2[4 * q + 1], v2 = pr2[4 * q + 2], v3 = pr2[4 * q + 3];
      const double pv[8] = {v0.x, v0.y, v1.x, v1.y, v2.x, v2.y, v3.x, v3.y};
      if (q == C / 8) {
        l = P[C] * (1.0 / pv[C % 8]);
        P[C] = l;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (8 * q + j > C) P[8 * q + j] -= l * pv[j];
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  pos = npos;
  if (tid == 0) piv[K0 + cr] = K0 + ppos;
}

template <int... Cs>
__device__ __attribute__((always_inline)) void own_columns(std::integer_sequence<int, Cs...>, double (&P)[kTB],
                                                           int& pos, int& singular, int gw, int g0r, int K0,
                                                           gint* __restrict__ piv, bool own, bool live,
                                                           gdouble* __restrict__ wrow, int nw, OwnLds& sh) {
  (own_column<Cs>(P, pos, singular, gw, g0r, K0, piv, own, live, wrow, nw, sh), ...);
}

// The rows r < m of the panel at positions >= plive take
// A[K0 + r, c0:c0+wt] -= A[K0 + r, g0:g0+kTB] U12 (U12 in sh.u.S), in
// 16-row strips per wavefront; CB = ceil(wt / 16) column blocks, a
// compile-time count so that the MFMA sequence has no branches.  Every load
// of a strip is issued at once; entries outside the block read A[0] and are
// never stored (each output entry depends only on its own input entry).
template <int CB>
__device__ __attribute__((always_inline)) void own_trailing(gdouble* __restrict__ A, int ld, int K0, int m, int g0,
                                                            int c0, int wt, int plive, OwnLds& sh) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = (int)blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll 1
  for (int rs = 16 * w; rs < m; rs += 16 * nw) {
    const bool aok = rs + li < m && sh.pos[rs + li] >= plive;
    if (__ballot(aok) == 0ull) continue;
    double a[kTB / 4];
#pragma unroll
    for (int ks = 0; ks < kTB / 4; ++ks) {
      const double v = A[aok ? (size_t)(K0 + rs + li) * ld + g0 + 4 * ks + lk : 0];
      a[ks] = aok ? -v : 0.0;
    }
    unsigned rmask = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = rs + 4 * v + lk;
      rmask |= (r < m && sh.pos[r] >= plive) ? (1u << v) : 0u;
    }
    const size_t cbase = (size_t)(K0 + rs + lk) * ld + c0 + li;
    dbl4 acc[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const bool ok = ((rmask >> v) & 1u) && 16 * cb + li < wt;
        acc[cb][v] = A[ok ? cbase + (size_t)(4 * v) * ld + 16 * cb : 0];
      }
#pragma unroll
    for (int ks = 0; ks < kTB / 4; ++ks) {
      double b[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) b[cb] = sh.u.S[4 * ks + lk][16 * cb + li];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], b[cb], acc[cb], 0, 0, 0);
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (((rmask >> v) & 1u) && 16 * cb + li < wt) A[cbase + (size_t)(4 * v) * ld + 16 * cb] = acc[cb][v];
  }
}

__device__ __attribute__((always_inline)) void panel_own_body(const GItem& it, int K0, OwnLds& sh) {
  gdouble* __restrict__ A = it.A;
  const int n = it.n, ld = it.ld;
  gwork* W = it.work;
  const int nthr = blockDim.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = nthr >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int m = n - K0, kb = lu_kb(n, K0);
  const bool own = tid < m;
  const gdouble* arow = A + (size_t)(K0 + (own ? tid : 0)) * ld;
  int pos = own ? tid : 0x7fff;
  int singular = 0;
#pragma unroll 1
  for (int gi = 0, g0r = 0; g0r < kb; ++gi, g0r += kTB) {
    const int gw = min(kTB, kb - g0r), g0 = K0 + g0r;
    const bool live = own && pos >= g0r;     // not pivoted in an earlier group
    // (rows not live and columns past gw hold values that are never used;
    // the address is clamped inside the row, the value not masked, so that
    // every load is in flight at once)
    double P[kTB];
#pragma unroll
    for (int c = 0; c < kTB; ++c) P[c] = arow[g0 + min(c, gw - 1)];
    gdouble* wrow = A + (size_t)(K0 + (own ? tid : 0)) * ld + g0;
    own_columns(std::make_integer_sequence<int, kTB>{}, P, pos, singular, gw, g0r, K0, it.piv, own, live, wrow, nw,
                sh);
    // the group's columns back in place, a row's 32 values together (a store
    // per finished column writes 8 bytes of a line at a time: several times
    // the bytes in HBM write traffic)
    if (live) {
#pragma unroll
      for (int c = 0; c < kTB; ++c)
        if (c < gw) wrow[c] = P[c];
    }
    __syncthreads();                         // the candidate rows are read; the LDS is reused
    // the group's pivot rows form the diagonal block, identity-padded beyond gw
    if (own && pos >= g0r && pos < g0r + gw) {
      const int i = pos - g0r;
#pragma unroll
      for (int c = 0; c < kTB; ++c) {
        const double v = c < gw ? P[c] : 0.0;
        sh.u.t.blk[i][c] = v;
        sh.u.t.inv2[kTB - 1 - i][kTB - 1 - c] = v;
      }
      sh.prow[i] = tid;
    }
    for (int idx = gw * kTB + tid; idx < kTB * kTB; idx += nthr) {
      const int i = idx >> 5, c = idx & 31;
      const double v = i == c ? 1.0 : 0.0;
      sh.u.t.blk[i][c] = v;
      sh.u.t.inv2[kTB - 1 - i][kTB - 1 - c] = v;
    }
    if (own) sh.pos[tid] = (short)pos;
    __syncthreads();
    own_block_inverses(gw, sh.u.t);
    for (int idx = tid; idx < kTB * kTB; idx += nthr) {
      it.uinv[(g0 / kTB) * kTB * kTB + idx] = sh.u.t.inv2[idx >> 5][idx & 31];
      W->inv[gi][idx >> 5][idx & 31] = sh.u.t.inv[idx >> 5][idx & 31];
    }
    __syncthreads();                         // the inverses are stored (E2 reads L11^-1 back)
    const int c0 = g0 + gw, wt = K0 + kb - c0;
    if (wt > 0) {
      // the pivot rows of the trailing columns ...
      for (int idx = tid; idx < kTB * kSW; idx += nthr) {
        const int i = idx / kSW, j = idx - i * kSW;
        sh.u.S[i][j] = (i < gw && j < wt) ? A[(size_t)(K0 + sh.prow[i]) * ld + c0 + j] : 0.0;
      }
      __syncthreads();
      // ... become U12 = L11^-1 A12 (in LDS and in place) ...
      const gdouble* __restrict__ linv = &W->inv[gi][0][0];
      for (int cb = 16 * w; cb < wt; cb += 16 * nw) {
        const int col = cb + li;
        const bool cok = col < wt;
        double xb[kTB / 4];
#pragma unroll
        for (int ks = 0; ks < kTB / 4; ++ks) xb[ks] = cok ? sh.u.S[4 * ks + lk][col] : 0.0;
        dbl4 acc[2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) acc[bi] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < kTB / 4; ++ks)
#pragma unroll
          for (int bi = 0; bi < 2; ++bi)
            acc[bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(linv[(16 * bi + li) * kTB + 4 * ks + lk], xb[ks], acc[bi],
                                                           0, 0, 0);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * bi + 4 * v + lk;
            if (cok && r < gw) {
              sh.u.S[r][col] = acc[bi][v];
              A[(size_t)(K0 + sh.prow[r]) * ld + c0 + col] = acc[bi][v];
            }
          }
      }
      __syncthreads();
      // ... and the rows not yet pivoted take A[r, c0:] -= L[r, group] U12
      // (a group with trailing columns is always kTB wide)
      const int CB = (wt + 15) >> 4;
      switch (CB) {
        case 1: own_trailing<1>(A, ld, K0, m, g0, c0, wt, g0r + gw, sh); break;
        case 2: own_trailing<2>(A, ld, K0, m, g0, c0, wt, g0r + gw, sh); break;
        case 3: own_trailing<3>(A, ld, K0, m, g0, c0, wt, g0r + gw, sh); break;
        case 4: own_trailing<4>(A, ld, K0, m, g0, c0, wt, g0r + gw, sh); break;
        case 5: own_trailing<5>(A, ld, K0, m, g0, c0, wt, g0r + gw, sh); break;
        default: own_trailing<6>(A, ld, K0, m, g0, c0, wt, g0r + gw, sh); break;
      }
      __syncthreads();
    }
  }
  // the rows that moved go to their positions, 32 columns at a time (every
  // read of a block precedes every write of it)
  const bool moved = own && pos != tid;
#pragma unroll 1
  for (int g0r = 0; g0r < kb; g0r += kTB) {
    const int gw = min(kTB, kb - g0r);
    double P[kTB];
    if (moved) {
#pragma unroll
      for (int c = 0; c < kTB; ++c) P[c] = arow[K0 + g0r + min(c, gw - 1)];
    }
    __syncthreads();
    if (moved) {
      gdouble* __restrict__ wr = A + (size_t)(K0 + pos) * ld + K0 + g0r;
#pragma unroll
      for (int c = 0; c < kTB; ++c)
        if (c < gw) wr[c] = P[c];
    }
  }
  // ... and so do their entries left of the panel (the step's interchanges
  // on L; only the tiles right of the panel are left to the U-row launches)
#pragma unroll 1
  for (int c0 = 0; c0 < K0; c0 += kTB) {
    const int cw = min(kTB, K0 - c0);
    double P[kTB];
    if (moved) {
#pragma unroll
      for (int c = 0; c < kTB; ++c) P[c] = arow[c0 + min(c, cw - 1)];
    }
    __syncthreads();
    if (moved) {
      gdouble* __restrict__ wr = A + (size_t)(K0 + pos) * ld + c0;
#pragma unroll
      for (int c = 0; c < kTB; ++c)
        if (c < cw) wr[c] = P[c];
    }
  }
  // the step's permutation for the other columns: row K0 + t receives the
  // old contents of row K0 + who[t]
  __syncthreads();                           // the LDS is reused
  if (own) sh.u.g.who[pos] = (short)tid;
  const unsigned long long mm = __ballot(moved);
  if (lane == 0) sh.u.g.wcount[w] = __popcll(mm);
  __syncthreads();
  int base = 0;
  for (int v = 0; v < w; ++v) base += sh.u.g.wcount[v];
  if (moved) sh.u.g.slot[tid] = (short)(base + __popcll(mm & ((1ull << lane) - 1ull)));
  __syncthreads();
  const int par = lu_step(n, K0) & 1;
  if (moved) {
    const int e = sh.u.g.slot[tid];
    W->rows[par][e] = K0 + tid;
    W->src[par][e] = sh.u.g.slot[sh.u.g.who[tid]];
  }
  if (tid == 0) {
    int total = 0;
    for (int v = 0; v < nw; ++v) total += sh.u.g.wcount[v];
    W->count[par] = total;
    if (K0 == 0 || singular) *it.status = singular;
  }
}

// One 16 x 16 output tile of alpha P Q (inner dimension K) by one wavefront
// on MFMA, operands read straight from global memory in the MFMA layouts:
// P(i, k) = p[i ld + k] for i < rows and k < cols, zero elsewhere (likewise
// Q).  p itself may point past the matrix: lanes outside the bounds read the
// valid address `safe` instead, so that every load is issued before the
// first product.  The tile is stored to c (leading dimension lc).
struct Opnd {
  const gdouble* p;
  int ld, rows, cols;
};

template <int K>
__device__ __attribute__((always_inline)) void wave_tile(Opnd P, Opnd Q, double alpha, gdouble* c, int lc,
                                                          const gdouble* safe) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  double a[K / 4], b[K / 4];
#pragma unroll
  for (int ks = 0; ks < K / 4; ++ks) {
    const int k = 4 * ks + lk;
    const bool pa = li < P.rows && k < P.cols, qa = k < Q.rows && li < Q.cols;
    const double va = *(pa ? P.p + li * P.ld + k : safe);
    const double vb = *(qa ? Q.p + k * Q.ld + li : safe);
    a[ks] = pa ? va : 0.0;
    b[ks] = qa ? vb : 0.0;
  }
  dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < K / 4; ++ks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], b[ks], acc, 0, 0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) c[(4 * v + lk) * lc + li] = alpha * acc[v];
}

// L11^-1 for the step's diagonal block (unit lower, kb x kb, zero-padded to
// kOuter x kOuter) from the stored inverses D_b of its 32 x 32 diagonal
// blocks, by doubling: a 2 x 2 block lower triangle [[P, 0], [C, Q]] has the
// inverse [[P^-1, 0], [-Q^-1 C P^-1, Q^-1]].  Five phases of MFMA tiles, the
// strictly upper blocks of the 128 x 128 result serving as scratch and
// cleared at the end:
//   0: X_bb = D_b, X_01 = X_23 = 0;   1: T_02 = L_10 D_0, T_03 = L_32 D_2;
//   2: X_10 = -D_1 T_02, X_32 = -D_3 T_03;
//   3: P = L[2:4, 0:2] X[0:2, 0:2] into X[0:2, 2:4];
//   4: X[2:4, 0:2] = -X[2:4, 2:4] P;   5: X[0:2, 2:4] = 0.
// Ends with a barrier.
__device__ __attribute__((always_inline)) void linv_body(const GItem& it, int K0) {
  const int n = it.n, ld = it.ld;
  gwork* W = it.work;
  gdouble* __restrict__ X = &W->linv[lu_step(n, K0) & 1][0][0];
  const int tid = threadIdx.x, w = tid >> 6;
  const int kb = lu_kb(n, K0);
  auto L = [&](int a, int b) {            // block (a, b), a > b, of L11
    return Opnd{it.A + (size_t)(K0 + kTB * a) * ld + K0 + kTB * b, ld, kb - kTB * a, kb - kTB * b};
  };
  auto D = [&](int b) {
    const int e = kTB * b < kb ? kTB : 0;
    return Opnd{&W->inv[b][0][0], kTB, e, e};
  };
  auto Xo = [&](int a, int b, int rows, int cols) {
    return Opnd{X + kTB * a * kOuter + kTB * b, kOuter, rows, cols};
  };
  auto at = [&](int a, int b) { return X + kTB * a * kOuter + kTB * b; };
  auto sub = [](Opnd o, int i, int k) {   // the 16 x 16 sub-tile (i, k) of an operand
    return Opnd{o.p + 16 * i * o.ld + 16 * k, o.ld, o.rows - 16 * i, o.cols - 16 * k};
  };
  // phase 0
  for (int idx = tid; idx < 4 * kTB * kTB; idx += kThreads) {
    const int b = idx >> 10, i = (idx >> 5) & 31, j = idx & 31;
    at(b, b)[i * kOuter + j] = kTB * b < kb ? W->inv[b][i][j] : 0.0;
  }
  for (int idx = tid; idx < 2 * kTB * kTB; idx += kThreads) {
    const int b = idx >> 10, i = (idx >> 5) & 31, j = idx & 31;
    at(2 * b, 2 * b + 1)[i * kOuter + j] = 0.0;
  }
  // phase 1: wavefront w takes product w / 4, output tile w % 4
  {
    const int pr = w >> 2, ti = (w >> 1) & 1, tj = w & 1;
    const Opnd Pm = pr ? L(3, 2) : L(1, 0), Qm = D(2 * pr);
    wave_tile<kTB>(sub(Pm, ti, 0), sub(Qm, 0, tj), 1.0, at(0, 2 + pr) + 16 * ti * kOuter + 16 * tj, kOuter, X);
  }
  __syncthreads();
  {
    const int pr = w >> 2, ti = (w >> 1) & 1, tj = w & 1;
    const Opnd Pm = D(2 * pr + 1), Qm = Xo(0, 2 + pr, kTB, kTB);
    wave_tile<kTB>(sub(Pm, ti, 0), sub(Qm, 0, tj), -1.0, at(2 * pr + 1, 2 * pr) + 16 * ti * kOuter + 16 * tj, kOuter,
                   X);
  }
  __syncthreads();
  // phases 3 and 4: 16 output tiles of 64 x 64, two per wavefront
  const Opnd L64 = Opnd{it.A + (size_t)(K0 + 2 * kTB) * ld + K0, ld, kb - 2 * kTB, kb};
  for (int t = w; t < 16; t += kThreads / kWave) {
    const int ti = t >> 2, tj = t & 3;
    wave_tile<2 * kTB>(sub(L64, ti, 0), sub(Xo(0, 0, 2 * kTB, 2 * kTB), 0, tj), 1.0,
                       at(0, 2) + 16 * ti * kOuter + 16 * tj, kOuter, X);
  }
  __syncthreads();
  for (int t = w; t < 16; t += kThreads / kWave) {
    const int ti = t >> 2, tj = t & 3;
    wave_tile<2 * kTB>(sub(Xo(2, 2, 2 * kTB, 2 * kTB), ti, 0), sub(Xo(0, 2, 2 * kTB, 2 * kTB), 0, tj), -1.0,
                       at(2, 0) + 16 * ti * kOuter + 16 * tj, kOuter, X);
  }
  __syncthreads();
  for (int idx = tid; idx < 2 * kTB * 2 * kTB; idx += kThreads) at(0, 2)[(idx >> 6) * kOuter + (idx & 63)] = 0.0;
  __syncthreads();
}

// Tile t of the step's U-row work.  LEFT: columns [128 t, ..) < K0 of L only
// take the step's interchanges.  Otherwise: columns K0 + kb + 128 t .. (the
// right-hand sides included) take the interchanges, are brought up to date
// with the long-K product against rows [K0, K0 + kb) of L -- which must
// already carry this step's interchanges, so the left tiles run in an earlier
// launch -- and become rows [K0, K0 + kb) of U.
template <bool LEFT>
__device__ __attribute__((always_inline)) void urow_body(const GItem& it, int K0, int t, MatLds& u,
                                                          PermLds& perm) {
  gdouble* A = it.A;
  const int n = it.n, ld = it.ld;
  const gwork* W = it.work;
  const int tid = threadIdx.x;
  const int kb = lu_kb(n, K0);
  // the last unit of the LEFT launch (the only one where the row-ownership
  // panel moved the rows left of it itself)
  if (LEFT && t == (it.cls <= 1 ? 0 : (K0 + kGT - 1) / kGT)) {
    linv_body(it, K0);
    return;
  }
  const int c0 = LEFT ? t * kGT : K0 + kb + t * kGT;
  const int c1 = min(LEFT ? K0 : ld, c0 + kGT);
  const int par = lu_step(n, K0) & 1;
  if (tid == 0) perm.count = W->count[par];
  for (int e = tid; e < 2 * kOuter; e += (int)blockDim.x) {
    perm.rows[e] = W->rows[par][e];
    perm.src[e] = W->src[par][e];
  }
  __syncthreads();
  apply_perm<LEFT ? kThreads : kGemmThreads>(A, ld, perm, c0, c1, 0, 0);
  if (LEFT) return;
  // the contributions of all earlier steps to these rows (left-looking: the
  // trailing matrix is never updated as a whole)
  if (K0 > 0) gemm_sub<kGemmThreads>(A, ld, K0, K0 + kb, c0, c1, 0, K0, u.g);
  // U12 = L11^-1 A12 as one MFMA product with the inverse the LEFT launch formed
  gemm_op<true, kGemmThreads>(A, ld, K0, K0 + kb, c0, c1, K0, K0 + kb, &W->linv[par][0][0], kOuter, K0, K0, u.g);
}

// Row tile t of the step's panel: the contributions of all earlier steps,
// A[K0 + 128 t .., K0 : K0 + kb] -= L[.., 0 : K0] U[0 : K0, K0 : K0 + kb].
__device__ __attribute__((always_inline)) void pupd_body(const GItem& it, int K0, int t, GemmLds& g) {
  const int n = it.n;
  const int kb = lu_kb(n, K0);
  const int ra = K0 + t * kGT;
  gemm_sub<kGemmThreads>(it.A, it.ld, ra, min(n, ra + kGT), K0, K0 + kb, 0, K0, g);
}

// Back substitution U W = R' on columns [n, n + nrhs), from the bottom in
// blocks of rows aligned with the factorisation's steps: the diagonal block is
// solved by its 32-row triangles (stored inverses on MFMA) and MFMA updates
// inside the block ...
// WIDE: right-hand sides beyond kGT columns (the updates inside the block
// then go through the tiled product, whose registers would otherwise halve
// the occupancy of the common case).
template <bool WIDE>
__device__ __attribute__((always_inline)) void bdiag_body(const GItem& it, int k0, MatLds& u) {
  gdouble* A = it.A;
  const int n = it.n, ld = it.ld, nrhs = it.nrhs;
  const int tid = threadIdx.x;
  const int k1 = k0 + lu_kb(n, k0);
  for (int a0 = k0 + (k1 - 1 - k0) / kTB * kTB; a0 >= k0; a0 -= kTB) {
    const int b1 = min(k1, a0 + kTB);
    for (int idx = tid; idx < kTB * kTB; idx += kThreads)
      u.t.inv[idx >> 5][idx & 31] = it.uinv[(a0 / kTB) * kTB * kTB + idx];
    __syncthreads();
    tri_apply<kTB>(A, ld, a0, b1 - a0, n, n + nrhs, u.t);
    if (a0 > k0) {
      // (the choice per matrix, not per batch, so that a matrix gets the same
      // bits in any batch)
      if (!WIDE || nrhs <= kGT) strip_update(A, ld, k0, a0, n, n + nrhs, a0, b1, u.g.Lt);
      else gemm_sub<kThreads>(A, ld, k0, a0, n, n + nrhs, a0, b1, u.g);
    }
  }
}

// ... after the contributions of every solved block below it are removed:
// R'[k0:k1] -= U[k0:k1, k1:n] W[k1:n] (left-looking: one long-K product per
// block instead of one short product per block above each solved one).
__device__ __attribute__((always_inline)) void bupd_body(const GItem& it, int k0, GemmLds& g) {
  const int n = it.n;
  const int k1 = k0 + lu_kb(n, k0);
  gemm_sub<kGemmThreads>(it.A, it.ld, k0, k1, n, n + it.nrhs, k1, n, g);
}

// ---------------------------------------------------------------------------
// Scheduled (persistent) kernels.  A work list is a prefix array pre[count+1]
// over the batch's matrices: matrix m owns global work indices
// [pre[m], pre[m+1]).  Each workgroup strides over the list, so one launch
// serves matrices of every size in the batch.

__device__ __forceinline__ int owner(const int32_t* __restrict__ pre, int count, int g) {
  int lo = 0, hi = count;                 // last m with pre[m] <= g
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// Work index of this workgroup in a flat launch.  Workgroups are dispatched
// to the 8 XCDs round-robin (workgroup b runs on XCD b mod 8), each with its
// own L2; the launch grid is padded to a multiple of 8 and XCD x takes the
// contiguous index range [x T8, (x + 1) T8), T8 = grid / 8, so the tiles of one
// matrix -- which share their L21 and U12 operands -- meet in one L2.
__device__ __forceinline__ int xcd_index() {
  const int t8 = (int)gridDim.x >> 3;
  return ((int)blockIdx.x & 7) * t8 + ((int)blockIdx.x >> 3);
}

__device__ __forceinline__ int back_block(const GItem& it, int step) {
  return lu_k0(it.n, lu_steps(it.n) - 1 - step);
}

// The register-panel kernel of the taller panels (orders above kOwnMax).
template <int ROWS, int NB>
__device__ __attribute__((always_inline)) void panel_launch(const LuItem* __restrict__ items,
                                                            const int32_t* __restrict__ pre, int count, int step,
                                                            PanelShared<NB>& sh) {
  const int gi = blockIdx.x;                 // one workgroup per matrix
  if (gi >= pre[count]) return;
  const int m = owner(pre, count, gi);
  panel_body<ROWS, NB>(gitem(items[m]), lu_k0(items[m].n, step), sh);
}

// Row-ownership panel: one workgroup per matrix, a thread per panel row
// (the launch's block size covers the tallest panel of the step).
__global__ __launch_bounds__(kOwnMax) void lu_panel_own_kernel(const LuItem* __restrict__ items,
                                                               const int32_t* __restrict__ pre, int count,
                                                               int step) {
  __shared__ __attribute__((aligned(16))) OwnLds sh;
  const int gi = blockIdx.x;                 // one workgroup per matrix
  if (gi >= pre[count]) return;
  const int m = owner(pre, count, gi);
  panel_own_body(gitem(items[m]), lu_k0(items[m].n, step), sh);
}

template <int ROWS, int NB>
__global__ __launch_bounds__(kThreads) void lu_panel_wide_kernel(const LuItem* __restrict__ items,
                                                                 const int32_t* __restrict__ pre, int count,
                                                                 int step) {
  __shared__ PanelShared<NB> sh;
  panel_launch<ROWS, NB>(items, pre, count, step, sh);
}

// PERSISTENT: each workgroup strides over the list; otherwise one workgroup
// per work unit (no loop, fewer live registers).
// OFF: the list's first unit is tile OFF of the matrix (the first tile and
// the rest of a step's U-row tiles are separate launches).
template <bool PERSISTENT, bool LEFT, int OFF = 0>
__global__ __launch_bounds__(LEFT ? kThreads : kGemmThreads) __attribute__((amdgpu_waves_per_eu(2))) void lu_urow_kernel(const LuItem* __restrict__ items,
                                                           const int32_t* __restrict__ pre, int count, int step) {
  __shared__ MatLds u;
  __shared__ PermLds perm;
  const int total = pre[count];
  if (!PERSISTENT) {
    const int gi = xcd_index();
    if (gi >= total) return;
    const int m = owner(pre, count, gi);
    urow_body<LEFT>(gitem(items[m]), lu_k0(items[m].n, step), gi - pre[m] + OFF, u, perm);
    return;
  }
  for (int gi = blockIdx.x; gi < total; gi += gridDim.x) {
    const int m = owner(pre, count, gi);
    urow_body<LEFT>(gitem(items[m]), lu_k0(items[m].n, step), gi - pre[m] + OFF, u, perm);
    __syncthreads();
  }
}

template <bool PERSISTENT>
__global__ __launch_bounds__(kGemmThreads) __attribute__((amdgpu_waves_per_eu(2))) void lu_pupd_kernel(
    const LuItem* __restrict__ items, const int32_t* __restrict__ pre, int count, int step) {
  __shared__ GemmLds g;
  const int total = pre[count];
  if (!PERSISTENT) {
    const int gi = xcd_index();
    if (gi >= total) return;
    const int m = owner(pre, count, gi);
    pupd_body(gitem(items[m]), lu_k0(items[m].n, step), gi - pre[m], g);
    return;
  }
  for (int gi = blockIdx.x; gi < total; gi += gridDim.x) {
    const int m = owner(pre, count, gi);
    pupd_body(gitem(items[m]), lu_k0(items[m].n, step), gi - pre[m], g);
  }
}

template <bool WIDE>
__global__ __launch_bounds__(kThreads) void lu_bdiag_kernel(const LuItem* __restrict__ items,
                                                            const int32_t* __restrict__ pre, int count, int step) {
  __shared__ MatLds u;
  const int gi = blockIdx.x;                 // one workgroup per matrix
  if (gi >= pre[count]) return;
  const GItem it = gitem(items[owner(pre, count, gi)]);
  bdiag_body<WIDE>(it, back_block(it, step), u);
}

template <bool PERSISTENT>
__global__ __launch_bounds__(kGemmThreads) __attribute__((amdgpu_waves_per_eu(2))) void lu_bupd_kernel(const LuItem* __restrict__ items,
                                                           const int32_t* __restrict__ pre, int count, int step) {
  __shared__ GemmLds g;
  const int total = pre[count];
  if (!PERSISTENT) {
    const int gi = xcd_index();
    if (gi >= total) return;
    const int m = owner(pre, count, gi);
    const GItem it = gitem(items[m]);
    bupd_body(it, back_block(it, step), g);
    return;
  }
  for (int gi = blockIdx.x; gi < total; gi += gridDim.x) {
    const int m = owner(pre, count, gi);
    const GItem it = gitem(items[m]);
    bupd_body(it, back_block(it, step), g);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side.

int lu_panel_class(int n) { return n <= 512 ? 0 : n <= 1024 ? 1 : n <= 2048 ? 2 : 3; }

size_t lu_work_bytes_per_matrix(int32_t n) {
  const size_t nblk = (size_t)(n + kTB - 1) / kTB;
  return sizeof(LuWork) + nblk * kTB * kTB * sizeof(double);
}

size_t lu_work_header_bytes() { return sizeof(LuWork); }

size_t lu_workspace_bytes(int32_t count, int32_t n) { return (size_t)count * lu_work_bytes_per_matrix(n); }

int lu_plan_tiles(const LuItem& it, int kind, int step) {
  const int n = it.n, ld = it.ld;
  const int nsteps = (n + kOuter - 1) / kOuter;
  if (step >= nsteps) return 0;
  const int K0 = lu_k0(n, step), kb = lu_kb(n, K0);
  switch (kind) {
    case LU_PANEL0: case LU_PANEL1: case LU_PANEL2: case LU_PANEL3:
      return it.cls == kind - LU_PANEL0 ? 1 : 0;
    case LU_LSWAP:      // the left tiles, then L11^-1 (the row-ownership panels move their rows' left part)
      return it.cls <= 1 ? 1 : (K0 + kGT - 1) / kGT + 1;
    case LU_UROW0: return (ld - K0 - kb + kGT - 1) / kGT > 0 ? 1 : 0;
    case LU_UREST: return std::max(0, (ld - K0 - kb + kGT - 1) / kGT - 1);
    case LU_PUPD: return K0 > 0 ? (n - K0 + kGT - 1) / kGT : 0;
    case LU_BDIAG: return 1;
    default: return step > 0 ? 1 : 0;           // LU_BUPD: the block (none for the bottom one)
  }
}

LuPlan::~LuPlan() {
  for (auto e : ev_main) (void)hipEventDestroy(e);
  for (auto e : ev_rest) (void)hipEventDestroy(e);
  if (side) (void)hipStreamDestroy(side);
}

void LuPlan::build(const std::vector<LuItem>& its) {
  items = its;
  count = (int32_t)its.size();
  wide_rhs = false;
  for (const auto& it : its) wide_rhs = wide_rhs || it.nrhs > kGT;
  nsteps = 0;
  for (const auto& it : its) nsteps = std::max(nsteps, (it.n + kOuter - 1) / kOuter);
  pre.assign((size_t)LU_KINDS * nsteps * (count + 1), 0);
  totals.assign((size_t)LU_KINDS * nsteps, 0);
  for (int kind = 0; kind < LU_KINDS; ++kind)
    for (int s = 0; s < nsteps; ++s) {
      int32_t* p = &pre[((size_t)kind * nsteps + s) * (count + 1)];
      p[0] = 0;
      for (int m = 0; m < count; ++m) p[m + 1] = p[m] + lu_plan_tiles(its[m], kind, s);
      totals[(size_t)kind * nsteps + s] = p[count];
    }
  // block size of the row-ownership panels: the step's tallest panel
  own_threads.assign((size_t)2 * nsteps, kWave);
  for (const auto& it : its)
    if (it.cls <= 1)
      for (int s = 0; s < lu_steps(it.n); ++s) {
        int32_t& t = own_threads[(size_t)it.cls * nsteps + s];
        t = std::max(t, (it.n - lu_k0(it.n, s) + kWave - 1) / kWave * kWave);
      }
  d_items.upload(items);
  d_pre.upload(pre);
  if (!side) PDD_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
  while ((int)ev_main.size() < nsteps) {
    hipEvent_t a, b;
    PDD_HIP(hipEventCreateWithFlags(&a, hipEventDisableTiming));
    PDD_HIP(hipEventCreateWithFlags(&b, hipEventDisableTiming));
    ev_main.push_back(a);
    ev_rest.push_back(b);
  }
}

int LuPlan::launch(hipStream_t st, int grid_cap, bool lookahead) const {
  const LuItem* di = d_items.ptr<LuItem>();
  int launches = 0;
  typedef void (*Kern)(const LuItem*, const int32_t*, int, int);
  // flat: one workgroup per unit; strided: a capped persistent grid
  auto go = [&](int kind, int s, Kern flat, Kern strided, hipStream_t q) {
    const int total = totals[(size_t)kind * nsteps + s];
    if (total == 0) return;
    const bool gemm = kind == LU_PUPD || kind == LU_UROW0 || kind == LU_UREST || kind == LU_BUPD;
    const int nthr = gemm ? kGemmThreads : kThreads;
    const int32_t* dp = d_pre.ptr<int32_t>() + ((size_t)kind * nsteps + s) * (count + 1);
    if (strided && grid_cap < total)
      hipLaunchKernelGGL(strided, dim3(grid_cap), dim3(nthr), 0, q, di, dp, count, s);
    else if (strided)   // flat tiled launch: grid padded to a multiple of the 8 XCDs
      hipLaunchKernelGGL(flat, dim3((total + 7) / 8 * 8), dim3(nthr), 0, q, di, dp, count, s);
    else
      hipLaunchKernelGGL(flat, dim3(total), dim3(nthr), 0, q, di, dp, count, s);
    ++launches;
  };
  // Look-ahead: the first U-row tile of step s (the columns of panel s + 1)
  // runs in order on st; the rest of the step's tiles run on the second stream
  // beside panel s + 1 and its pre-update and interchanges, which touch
  // other columns.  The first tile of step s + 1 waits for them (it covers
  // columns they bring up to date).
  int rest = -1;
  for (int s = 0; s < nsteps; ++s) {
    go(LU_PUPD, s, lu_pupd_kernel<false>, lu_pupd_kernel<true>, st);
    for (int kind = LU_PANEL0; kind <= LU_PANEL1; ++kind) {
      const int total = totals[(size_t)kind * nsteps + s];
      if (total == 0) continue;
      const int32_t* dp = d_pre.ptr<int32_t>() + ((size_t)kind * nsteps + s) * (count + 1);
      hipLaunchKernelGGL(lu_panel_own_kernel, dim3(total), dim3(own_threads[(size_t)(kind - LU_PANEL0) * nsteps + s]),
                         0, st, di, dp, count, s);
      ++launches;
    }
    go(LU_PANEL2, s, lu_panel_wide_kernel<4, 16>, nullptr, st);
    go(LU_PANEL3, s, lu_panel_wide_kernel<8, 8>, nullptr, st);
    go(LU_LSWAP, s, lu_urow_kernel<false, true>, lu_urow_kernel<true, true>, st);
    if (rest >= 0) PDD_HIP(hipStreamWaitEvent(st, ev_rest[rest], 0));
    rest = -1;
    go(LU_UROW0, s, lu_urow_kernel<false, false, 0>, lu_urow_kernel<true, false, 0>, st);
    if (!lookahead) {
      go(LU_UREST, s, lu_urow_kernel<false, false, 1>, lu_urow_kernel<true, false, 1>, st);
    } else if (totals[(size_t)LU_UREST * nsteps + s] > 0) {
      PDD_HIP(hipEventRecord(ev_main[s], st));
      PDD_HIP(hipStreamWaitEvent(side, ev_main[s], 0));
      go(LU_UREST, s, lu_urow_kernel<false, false, 1>, lu_urow_kernel<true, false, 1>, side);
      PDD_HIP(hipEventRecord(ev_rest[s], side));
      rest = s;
    }
  }
  if (rest >= 0) PDD_HIP(hipStreamWaitEvent(st, ev_rest[rest], 0));
  for (int s = 0; s < nsteps; ++s) {
    go(LU_BUPD, s, lu_bupd_kernel<false>, lu_bupd_kernel<true>, st);
    go(LU_BDIAG, s, wide_rhs ? lu_bdiag_kernel<true> : lu_bdiag_kernel<false>, nullptr, st);
  }
  return launches;
}

int launch_lu_solve(const BucketTables& T, int32_t count, double* A, int64_t mat_stride,
                    int32_t* piv, int32_t* status, void* work, hipStream_t st) {
  std::vector<LuItem> its(count);
  char* w = static_cast<char*>(work);
  const size_t per = lu_work_bytes_per_matrix(T.n);
  for (int m = 0; m < count; ++m) {
    LuItem& it = its[m];
    it.A = A + (int64_t)m * mat_stride;
    it.piv = piv + (int64_t)m * T.n;
    it.status = status + m;
    it.work = reinterpret_cast<LuWork*>(w + m * per);
    it.uinv = reinterpret_cast<double*>(w + m * per + sizeof(LuWork));
    it.n = T.n;
    it.ld = T.ld;
    it.nrhs = T.nrhs;
    it.cls = lu_panel_class(T.n);
  }
  LuPlan plan;
  plan.build(its);
  const int launches = plan.launch(st, 1 << 30);
  PDD_HIP(hipStreamSynchronize(st));     // the plan's device lists are freed on return
  return launches;
}

}  // namespace pdd
