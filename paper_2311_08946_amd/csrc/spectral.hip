// Floating rows of C and r on gfx950: polar Chebyshev x Fourier collocation of
// the local problems (Section 2.4 eqs. 31-35, Section 3.3 eqs. 40-41), batched
// LU with partial pivoting on FP64 MFMA, back substitution, interpolation at
// the assigned knots and scatter into the CSR values.
//
// Matrix layout (one per floating circle, row-major, leading dimension ld):
//   columns [0, n)        A_II, the collocation rows at the n interior nodes
//   columns [n, n+M)      A_IB H, ring columns mapped onto the M knot values
//   column  n+M           -F
//   columns [n+M+1, ld)   zero padding
// Each row is scaled by 1 / max_j |A_II[q, j]| (row equilibration).  After the
// LU, columns [n, n+M+1) hold W = A_II^-1 [A_IB H | -F].
#include "kernels.h"

namespace pdd {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

}  // namespace

// ------------------------------------------------------------------ sampling

__global__ __launch_bounds__(256) void sample_nodes_kernel(const DevProblem* __restrict__ P,
                                                           BucketTables T, ChunkDesc C,
                                                           double* o0, double* o1, double* o2,
                                                           double* o3, double* o4, double* o5,
                                                           double* o6) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= T.n) return;
  const int f = C.fl[blockIdx.y];
  const int m = C.float_ids[f];
  const int jr = q / T.Nt + 1;
  const int l = q - (jr - 1) * T.Nt;
  const double rr = C.rad[m] * T.xr[jr];
  const double x = C.cx[m] + rr * T.cs[l];
  const double y = C.cy[m] + rr * T.sn[l];
  double co[7];
  coefficients_at(*P, x, y, co);
  const int64_t node = C.node_off[f] + q;
  double* outs[7] = {o0, o1, o2, o3, o4, o5, o6};
#pragma unroll
  for (int t = 0; t < 7; ++t)
    if (outs[t]) outs[t][node] = co[t];
}

void launch_sample_nodes(const DevProblem* P, const BucketTables& T, const ChunkDesc& C,
                         double* const out[7], hipStream_t st) {
  dim3 grid((T.n + 255) / 256, C.count);
  hipLaunchKernelGGL(sample_nodes_kernel, grid, dim3(256), 0, st, P, T, C, out[0], out[1],
                     out[2], out[3], out[4], out[5], out[6]);
}

// ------------------------------------------------------- K1: collocation rows

// One wavefront per row.  Row q = (jr - 1) Ntheta + l is the polar form of
//   a_xx/2 u_xx + a_xy u_xy + a_yy/2 u_yy + b_x u_x + b_y u_y + c u
// at radius rho = x_jr, angle theta_l, on a circle of radius r, with
// derivatives taken on the full diameter grid and folded onto the unknowns by
// u(-rho, theta) = u(rho, theta + pi).
__global__ __launch_bounds__(256) void colloc_build_kernel(BucketTables T, ChunkDesc C,
                                                           NodeSamples S, double* __restrict__ A,
                                                           int64_t stride,
                                                           double* __restrict__ rowscale) {
  extern __shared__ double s_ring[];          // [4][Nt] scaled A_IB rows
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = T.n, Nt = T.Nt, Nc = T.Nc, M = T.M, ld = T.ld;
  const int ci = blockIdx.y;
  const int f = C.fl[ci];
  const int m = C.float_ids[f];
  const int q = blockIdx.x * 4 + w;
  const bool active = q < n;
  const int qq = active ? q : 0;
  const int jr = qq / Nt + 1;
  const int l = qq - (jr - 1) * Nt;
  const int64_t node = C.node_off[f] + qq;
  const double axx = S.s[0][node], axy = S.s[1][node], ayy = S.s[2][node];
  const double bx = S.s[3][node], by = S.s[4][node], cc = S.s[5][node], ff = S.s[6][node];
  const double r = C.rad[m];
  const double rho = T.xr[jr];
  const double cth = T.cs[l], sth = T.sn[l];
  const double r2 = r * r;
  const double ss = sth * sth, cc2 = cth * cth, sc = sth * cth, c2s2 = cc2 - ss;
  // coefficients of u_rho_rho, u_rho, u_theta_theta, u_rho_theta, u_theta
  const double c_rr = (0.5 * axx * cc2 + axy * sc + 0.5 * ayy * ss) / r2;
  const double ang = 0.5 * axx * ss - axy * sc + 0.5 * ayy * cc2;
  const double c_r = ang / (rho * r2) + (bx * cth + by * sth) / r;
  const double c_tt = ang / (rho * rho * r2);
  const double c_rt = (-axx * sc + axy * c2s2 + ayy * sc) / (rho * r2);
  const double c_t = (axx * sc - axy * c2s2 - ayy * sc) / (rho * rho * r2) +
                     (-bx * sth + by * cth) / (rho * r);
  const double* Drow = T.Dr + (int64_t)(jr - 1) * (Nc + 1);
  const double* D2row = T.D2r + (int64_t)(jr - 1) * (Nc + 1);
  const int half = Nt / 2;

  // full-grid operator entry at radial index j, angular index lp
  auto entry = [&](int j, int lp) -> double {
    int dl = l - lp;
    if (dl < 0) dl += Nt;
    const double dj = Drow[j];
    double v = c_rt * dj * T.d1t[dl];
    if (lp == l) v += c_rr * D2row[j] + c_r * dj;
    if (j == jr) v += c_tt * T.d2t[dl] + c_t * T.d1t[dl];
    return v;
  };
  auto interior = [&](int col) -> double {
    const int k = col / Nt + 1;
    const int lp = col - (k - 1) * Nt;
    int lq = lp - half;
    if (lq < 0) lq += Nt;
    double v = entry(k, lp) + entry(Nc - k, lq);
    if (col == qq) v += cc;
    return v;
  };
  auto ring = [&](int lp) -> double {
    int lq = lp - half;
    if (lq < 0) lq += Nt;
    return entry(0, lp) + entry(Nc, lq);
  };

  double mx = 0.0;
  for (int col = lane; col < n; col += kWave) mx = fmax(mx, fabs(interior(col)));
  mx = wave_max(mx);
  const double scale = 1.0 / mx;
  double* row = A + (int64_t)ci * stride + (int64_t)qq * ld;
  if (active) {
    if (lane == 0) rowscale[(int64_t)ci * n + q] = scale;
    for (int col = lane; col < n; col += kWave) row[col] = scale * interior(col);
    for (int lp = lane; lp < Nt; lp += kWave) s_ring[w * Nt + lp] = scale * ring(lp);
  }
  __syncthreads();
  if (active) {
    for (int j = lane; j < M; j += kWave) {
      double v = 0.0;
      for (int lp = 0; lp < Nt; ++lp) v += s_ring[w * Nt + lp] * T.H[(int64_t)lp * M + j];
      row[n + j] = v;
    }
    if (lane == 0) row[n + M] = -scale * ff;
    for (int col = n + M + 1 + lane; col < ld; col += kWave) row[col] = 0.0;
  }
}

void launch_colloc_build(const BucketTables& T, const ChunkDesc& C, const NodeSamples& S,
                         double* A, int64_t mat_stride, double* rowscale, hipStream_t st) {
  dim3 grid((T.n + 3) / 4, C.count);
  size_t shm = sizeof(double) * 4 * T.Nt;
  hipLaunchKernelGGL(colloc_build_kernel, grid, dim3(256), shm, st, T, C, S, A, mat_stride,
                     rowscale);
}

// ----------------------------------------------------------------- K2: LU

// One workgroup (8 wavefronts) factorises one matrix, right-looking with a
// panel of NB columns.  The panel is held in registers (thread t owns rows
// k0 + t + 512 s), factorised column by column with a workgroup-wide pivot
// search; its row interchanges are then applied to the remaining columns, the
// block row of U is formed by a triangular solve, and the trailing matrix
// (including the right-hand-side columns) is updated on FP64 MFMA
// (v_mfma_f64_16x16x4: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
// D[i][j] in register v of lane j + 16 (i mod 4) with v = i / 4).
namespace {

constexpr int kLuThreads = 512;
constexpr int kTileR = 128;    // trailing tile rows (4 x 32 per wave group)
constexpr int kTileC = 64;     // trailing tile cols (2 x 32)

typedef double dbl4 __attribute__((ext_vector_type(4)));

template <int NB>
__device__ __forceinline__ void trailing_update(double* __restrict__ A, int ld, int n, int k0,
                                                double (*s_Lt)[kTileR + 4],
                                                double (*s_Ut)[kTileC + 4]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int R0 = k0 + NB;
  for (int rb = R0; rb < n; rb += kTileR) {
    // L21 band, transposed into LDS
    for (int idx = tid; idx < kTileR * NB; idx += kLuThreads) {
      const int i = idx / NB, k = idx - i * NB;
      const int row = rb + i;
      s_Lt[k][i] = (row < n) ? -A[(int64_t)row * ld + k0 + k] : 0.0;
    }
    for (int cb = R0; cb < ld; cb += kTileC) {
      for (int idx = tid; idx < NB * kTileC; idx += kLuThreads) {
        const int k = idx / kTileC, j = idx - k * kTileC;
        const int col = cb + j;
        s_Ut[k][j] = (col < ld) ? A[(int64_t)(k0 + k) * ld + col] : 0.0;
      }
      __syncthreads();
      dbl4 acc[2][2];
      const int rbase = rb + 32 * wr, cbase = cb + 32 * wc;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = rbase + 16 * bi + 4 * v + (lane >> 4);
            const int col = cbase + 16 * bj + (lane & 15);
            acc[bi][bj][v] = (row < n && col < ld) ? A[(int64_t)row * ld + col] : 0.0;
          }
#pragma unroll
      for (int ks = 0; ks < NB / 4; ++ks) {
        const int kr = 4 * ks + (lane >> 4);
        double a[2], b[2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) a[bi] = s_Lt[kr][32 * wr + 16 * bi + (lane & 15)];
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) b[bj] = s_Ut[kr][32 * wc + 16 * bj + (lane & 15)];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
            acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
      }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = rbase + 16 * bi + 4 * v + (lane >> 4);
            const int col = cbase + 16 * bj + (lane & 15);
            if (row < n && col < ld) A[(int64_t)row * ld + col] = acc[bi][bj][v];
          }
      __syncthreads();
    }
  }
}

template <int ROWS, int NB>
__global__ __launch_bounds__(kLuThreads) void lu_kernel(double* __restrict__ A0, int n, int ld,
                                                        int64_t stride, int32_t* __restrict__ piv0,
                                                        int32_t* __restrict__ status) {
  __shared__ double s_prow[NB], s_krow[NB];
  __shared__ double s_L11[NB][NB + 1];
  __shared__ double s_redv[kLuThreads / 64];
  __shared__ int s_redi[kLuThreads / 64];
  __shared__ int s_piv[NB];
  __shared__ double s_Lt[NB][kTileR + 4];
  __shared__ double s_Ut[NB][kTileC + 4];

  double* A = A0 + (int64_t)blockIdx.x * stride;
  int32_t* piv = piv0 + (int64_t)blockIdx.x * n;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int singular = 0;
  double P[ROWS][NB];

  for (int k0 = 0; k0 < n; k0 += NB) {
    const int pw = min(NB, n - k0);
#pragma unroll
    for (int s = 0; s < ROWS; ++s) {
      const int row = k0 + tid + kLuThreads * s;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        P[s][c] = (row < n && c < pw) ? A[(int64_t)row * ld + k0 + c] : 0.0;
    }
#pragma unroll 1
    for (int c = 0; c < pw; ++c) {
      const int kk = k0 + c;
      // column c of the owned rows (register arrays are indexed statically)
      double colv[ROWS];
#pragma unroll
      for (int s = 0; s < ROWS; ++s) {
        double v = 0.0;
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) v = (cc == c) ? P[s][cc] : v;
        colv[s] = v;
      }
      // pivot search: largest |a|, smallest row on ties
      double bv = -1.0;
      int bi = 0x7fffffff;
#pragma unroll
      for (int s = 0; s < ROWS; ++s) {
        const int row = k0 + tid + kLuThreads * s;
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
      for (int t = 1; t < kLuThreads / 64; ++t) {
        const double ov = s_redv[t];
        const int oi = s_redi[t];
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      }
      const int p = (bv > 0.0) ? bi : kk;
      if (!(bv > 0.0)) singular = 1;
      // interchange rows kk and p inside the panel (owners exchange via LDS)
      const int tp = (p - k0) & (kLuThreads - 1), sp = (p - k0) / kLuThreads;
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
          const int row = k0 + tid + kLuThreads * s;
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
        s_piv[c] = p;
        piv[kk] = p;
      }
      __syncthreads();
    }
    // panel back to memory
#pragma unroll
    for (int s = 0; s < ROWS; ++s) {
      const int row = k0 + tid + kLuThreads * s;
      if (row < n)
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c < pw) A[(int64_t)row * ld + k0 + c] = P[s][c];
    }
    // the panel's interchanges on every other column (each thread owns columns)
    for (int col = tid; col < ld; col += kLuThreads) {
      if (col >= k0 && col < k0 + pw) continue;
      for (int c = 0; c < pw; ++c) {
        const int p = s_piv[c];
        const int kk = k0 + c;
        if (p != kk) {
          const double t0 = A[(int64_t)kk * ld + col];
          A[(int64_t)kk * ld + col] = A[(int64_t)p * ld + col];
          A[(int64_t)p * ld + col] = t0;
        }
      }
    }
    if (tid < pw) {
#pragma unroll
      for (int c = 0; c < NB; ++c) s_L11[tid][c] = P[0][c];
    }
    __syncthreads();
    // block row of U: L11^-1 A12 (unit lower triangular)
    for (int col = k0 + pw + tid; col < ld; col += kLuThreads) {
      double x[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = (c < pw) ? A[(int64_t)(k0 + c) * ld + col] : 0.0;
#pragma unroll 1
      for (int c = 1; c < pw; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int c2 = 0; c2 < NB; ++c2) acc += (c2 < c) ? s_L11[c][c2] * x[c2] : 0.0;
#pragma unroll
        for (int c3 = 0; c3 < NB; ++c3) x[c3] = (c3 == c) ? x[c3] - acc : x[c3];
      }
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < pw) A[(int64_t)(k0 + c) * ld + col] = x[c];
    }
    __syncthreads();
    if (k0 + NB < n) trailing_update<NB>(A, ld, n, k0, s_Lt, s_Ut);
    __syncthreads();
  }
  if (tid == 0) status[blockIdx.x] = singular;
  (void)lane;
}

}  // namespace

void launch_lu(const BucketTables& T, int32_t count, double* A, int64_t mat_stride,
               int32_t* piv, int32_t* status, hipStream_t st) {
  const int n = T.n;
  if (n <= 512)
    hipLaunchKernelGGL((lu_kernel<1, 32>), dim3(count), dim3(kLuThreads), 0, st, A, n, T.ld,
                       mat_stride, piv, status);
  else if (n <= 1024)
    hipLaunchKernelGGL((lu_kernel<2, 32>), dim3(count), dim3(kLuThreads), 0, st, A, n, T.ld,
                       mat_stride, piv, status);
  else if (n <= 2048)
    hipLaunchKernelGGL((lu_kernel<4, 16>), dim3(count), dim3(kLuThreads), 0, st, A, n, T.ld,
                       mat_stride, piv, status);
  else
    hipLaunchKernelGGL((lu_kernel<8, 8>), dim3(count), dim3(kLuThreads), 0, st, A, n, T.ld,
                       mat_stride, piv, status);
}

// ------------------------------------------------------ K3: back substitution

// U W = R' on the right-hand-side columns, 32-row blocks from the bottom: the
// block is first reduced by the rows already solved, then solved by one
// thread per right-hand side.
__global__ __launch_bounds__(512) void backsolve_kernel(double* __restrict__ A0, int n, int ld,
                                                        int nrhs, int64_t stride) {
  constexpr int BR = 32;
  double* A = A0 + (int64_t)blockIdx.x * stride;
  const int tid = threadIdx.x;
  const int i = tid >> 4;         // row in block (0..31)
  const int cg = tid & 15;        // column group
  for (int k1 = n; k1 > 0; k1 -= BR) {
    const int k0 = max(0, k1 - BR);
    if (k0 + i < k1) {
      const double* urow = A + (int64_t)(k0 + i) * ld;
      double acc[9];
#pragma unroll
      for (int u = 0; u < 9; ++u) acc[u] = 0.0;
      for (int q = k1; q < n; ++q) {
        const double uv = urow[q];
        const double* wrow = A + (int64_t)q * ld + n;
#pragma unroll
        for (int u = 0; u < 9; ++u) {
          const int c = cg + 16 * u;
          if (c < nrhs) acc[u] += uv * wrow[c];
        }
      }
#pragma unroll
      for (int u = 0; u < 9; ++u) {
        const int c = cg + 16 * u;
        if (c < nrhs) A[(int64_t)(k0 + i) * ld + n + c] -= acc[u];
      }
    }
    __syncthreads();
    for (int c = tid; c < nrhs; c += 512) {
      for (int r = k1 - 1; r >= k0; --r) {
        const double* urow = A + (int64_t)r * ld;
        double x = urow[n + c];
        for (int q = r + 1; q < k1; ++q) x -= urow[q] * A[(int64_t)q * ld + n + c];
        A[(int64_t)r * ld + n + c] = x / urow[r];
      }
    }
    __syncthreads();
  }
}

void launch_backsolve(const BucketTables& T, int32_t count, double* A, int64_t mat_stride,
                      hipStream_t st) {
  hipLaunchKernelGGL(backsolve_kernel, dim3(count), dim3(512), 0, st, A, T.n, T.ld, T.nrhs,
                     mat_stride);
}

// ------------------------------------------- K4: knot evaluation and scatter

// One workgroup per floating circle.  For each assigned knot (rho*, phi*), the
// interpolation weights over the full diameter grid are barycentric Lagrange
// weights in rho times Ntheta-point periodic cardinals in theta; folded onto
// the unknowns they give e (interior) and eps (ring):
//   C[i, Xi_m] = e^T W[:, :M] - eps^T H,   r_i = e^T W[:, M],   C_ii = 1.
namespace {
constexpr int kEvalKnots = 32;
constexpr int kEvalGroups = 8;    // 256 threads = 32 knots x 8 column groups
constexpr int kEvalQ = 32;
constexpr int kEvalMaxPer = 17;   // columns per thread: nrhs <= 136
}

__global__ __launch_bounds__(256) void eval_scatter_kernel(BucketTables T, ChunkDesc C,
                                                           const double* __restrict__ A0,
                                                           int64_t stride, double* __restrict__ val,
                                                           double* __restrict__ bvec) {
  extern __shared__ double sh[];
  const int Nc1 = T.Nc + 1, Nt = T.Nt, n = T.n, M = T.M, nrhs = T.nrhs, ld = T.ld;
  double* lx = sh;                                  // [kEvalKnots][Nc+1]
  double* lt = lx + kEvalKnots * Nc1;               // [kEvalKnots][Nt]
  double* Ws = lt + kEvalKnots * Nt;                // [kEvalQ][nrhs]
  const int tid = threadIdx.x;
  const int ci = blockIdx.x;
  const int f = C.fl[ci];
  const int m = C.float_ids[f];
  const double* A = A0 + (int64_t)ci * stride;
  const int64_t klo = C.fk_off[f], khi = C.fk_off[f + 1];
  const double cxm = C.cx[m], cym = C.cy[m], rm = C.rad[m];
  const int half = Nt / 2;
  const int t = tid & (kEvalKnots - 1), cg = tid / kEvalKnots;
  for (int64_t base = klo; base < khi; base += kEvalKnots) {
    const int cnt = (int)min<int64_t>(kEvalKnots, khi - base);
    if (tid < cnt) {
      const int i = C.fk_ids[base + tid];
      const double dx = C.kx[i] - cxm, dy = C.ky[i] - cym;
      const double rho = sqrt(dx * dx + dy * dy) / rm;
      const double phi = atan2(dy, dx);
      int exact = -1;
      double ssum = 0.0;
      for (int j = 0; j < Nc1; ++j) {
        const double d = rho - T.xr[j];
        if (d == 0.0) exact = j;
        else ssum += T.bw[j] / d;
      }
      for (int j = 0; j < Nc1; ++j)
        lx[tid * Nc1 + j] = (exact >= 0) ? (j == exact ? 1.0 : 0.0)
                                         : (T.bw[j] / (rho - T.xr[j])) / ssum;
      const double hstep = kTwoPiD / Nt;
      for (int l = 0; l < Nt; ++l) {
        const double x = 0.5 * (phi - hstep * l);
        double sx, cx;
        sincos(x, &sx, &cx);
        // periodic cardinal sin(Nt x) cos(x) / (Nt sin(x)) at half-angle x
        lt[tid * Nt + l] = (fabs(sx) < 1e-15) ? 1.0 : sin(Nt * x) * cx / (Nt * sx);
      }
    }
    __syncthreads();
    double acc[kEvalMaxPer];
#pragma unroll
    for (int u = 0; u < kEvalMaxPer; ++u) acc[u] = 0.0;
    for (int q0 = 0; q0 < n; q0 += kEvalQ) {
      const int qn = min(kEvalQ, n - q0);
      for (int idx = tid; idx < qn * nrhs; idx += 256) {
        const int qq = idx / nrhs, c = idx - qq * nrhs;
        Ws[qq * nrhs + c] = A[(int64_t)(q0 + qq) * ld + n + c];
      }
      __syncthreads();
      if (t < cnt) {
        for (int qq = 0; qq < qn; ++qq) {
          const int q = q0 + qq;
          const int k = q / Nt + 1;
          const int lp = q - (k - 1) * Nt;
          int lq = lp + half;
          if (lq >= Nt) lq -= Nt;
          const double e = lx[t * Nc1 + k] * lt[t * Nt + lp] + lx[t * Nc1 + (Nc1 - 1 - k)] * lt[t * Nt + lq];
#pragma unroll
          for (int u = 0; u < kEvalMaxPer; ++u) {
            const int c = cg + kEvalGroups * u;
            if (c < nrhs) acc[u] += e * Ws[qq * nrhs + c];
          }
        }
      }
      __syncthreads();
    }
    if (t < cnt) {
      for (int l = 0; l < Nt; ++l) {
        int lq = l + half;
        if (lq >= Nt) lq -= Nt;
        const double eps = lx[t * Nc1] * lt[t * Nt + l] + lx[t * Nc1 + Nc1 - 1] * lt[t * Nt + lq];
#pragma unroll
        for (int u = 0; u < kEvalMaxPer; ++u) {
          const int c = cg + kEvalGroups * u;
          if (c < M) acc[u] -= eps * T.H[(int64_t)l * M + c];
        }
      }
      const int i = C.fk_ids[base + t];
      const int64_t lo = C.knot_off[m];
      const int64_t p = C.rowptr[i];
      const int shift = (i < lo) ? 1 : 0;
#pragma unroll
      for (int u = 0; u < kEvalMaxPer; ++u) {
        const int c = cg + kEvalGroups * u;
        if (c < M) val[p + shift + c] = acc[u];
        else if (c == M) bvec[i] = acc[u];
      }
      if (cg == 0) val[p + (shift ? 0 : M)] = 1.0;
    }
    __syncthreads();
  }
}

void launch_eval_scatter(const BucketTables& T, const ChunkDesc& C, const double* A,
                         int64_t mat_stride, double* val, double* b, hipStream_t st) {
  size_t shm = sizeof(double) * ((size_t)kEvalKnots * (T.Nc + 1 + T.Nt) + (size_t)kEvalQ * T.nrhs);
  hipLaunchKernelGGL(eval_scatter_kernel, dim3(C.count), dim3(256), shm, st, T, C, A, mat_stride,
                     val, b);
}

}  // namespace pdd
