// Floating rows of C and r on gfx950: polar Chebyshev x Fourier collocation of
// the local problems (Section 2.4 eqs. 31-35, Section 3.3 eqs. 40-41),
// interpolation of the local solutions at the assigned knots and scatter into
// the CSR values.  The batched LU and back substitution are in lu.hip.
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
// u(-rho, theta) = u(rho, theta + pi).  The row is assembled once in LDS (the
// wavefront's own slice) and then scaled and written with coalesced stores.
// Without the mixed term (a_xy = 0 and a_xx = a_yy, so u_rho_theta drops out)
// only the radial line (angle theta_l and its opposite) and the angular ring
// (radius x_jr) are non-zero: 2 Nr + Ntheta entries instead of n.
namespace {
constexpr int kBuildWaves = 4;

// Orders the wavefront's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
}  // namespace

__global__ __launch_bounds__(256) void colloc_build_kernel(BucketTables T, ChunkDesc C,
                                                           NodeSamples S, double* __restrict__ A,
                                                           int64_t stride,
                                                           double* __restrict__ rowscale) {
  extern __shared__ double s_build[];          // per wavefront: row [n], ring [Nt]
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = T.n, Nt = T.Nt, Nc = T.Nc, Nr = T.Nr, M = T.M, ld = T.ld;
  double* s_row = s_build + (int64_t)w * (n + Nt);
  double* s_ring = s_row + n;
  const int ci = blockIdx.y;
  const int f = C.fl[ci];
  const int m = C.float_ids[f];
  const int q = blockIdx.x * kBuildWaves + w;
  if (q >= n) return;                          // no workgroup barrier below
  const int jr = q / Nt + 1;
  const int l = q - (jr - 1) * Nt;
  const int64_t node = C.node_off[f] + q;
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
  const bool mixed = !(axy == 0.0 && axx == ayy);
  const double c_rt = mixed ? (-axx * sc + axy * c2s2 + ayy * sc) / (rho * r2) : 0.0;
  const double c_t = (axx * sc - axy * c2s2 - ayy * sc) / (rho * rho * r2) +
                     (-bx * sth + by * cth) / (rho * r);
  const double* Drow = T.Dr + (int64_t)(jr - 1) * (Nc + 1);
  const double* D2row = T.D2r + (int64_t)(jr - 1) * (Nc + 1);
  const int half = Nt / 2;

  if (mixed) {
    // dense: every full-grid entry, folded
    auto entry = [&](int j, int lp) -> double {
      int dl = l - lp;
      if (dl < 0) dl += Nt;
      const double dj = Drow[j];
      double v = c_rt * dj * T.d1t[dl];
      if (lp == l) v += c_rr * D2row[j] + c_r * dj;
      if (j == jr) v += c_tt * T.d2t[dl] + c_t * T.d1t[dl];
      return v;
    };
    for (int col = lane; col < n; col += kWave) {
      const int k = col / Nt + 1;
      const int lp = col - (k - 1) * Nt;
      int lq = lp - half;
      if (lq < 0) lq += Nt;
      s_row[col] = entry(k, lp) + entry(Nc - k, lq);
    }
    for (int lp = lane; lp < Nt; lp += kWave) {
      int lq = lp - half;
      if (lq < 0) lq += Nt;
      s_ring[lp] = entry(0, lp) + entry(Nc, lq);
    }
  } else {
    for (int col = lane; col < n; col += kWave) s_row[col] = 0.0;
    for (int lp = lane; lp < Nt; lp += kWave) s_ring[lp] = 0.0;
    wave_sync();
    // radial line: full-grid index j at angle theta_l; j in [1, Nr] is the
    // interior node (j, l), j in [Nr + 1, Nc - 1] folds to (Nc - j, l + half),
    // j = 0 and j = Nc are the ring at l and l + half
    const int lh = (l + half) % Nt;
    for (int j = lane; j <= Nc; j += kWave) {
      const double v = c_rr * D2row[j] + c_r * Drow[j];
      if (j == 0) s_ring[l] += v;
      else if (j == Nc) s_ring[lh] += v;
      else if (j <= Nr) s_row[(j - 1) * Nt + l] += v;
      else s_row[(Nc - j - 1) * Nt + lh] += v;
    }
    wave_sync();
    // angular ring at radius x_jr (interior row jr only)
    for (int lp = lane; lp < Nt; lp += kWave) {
      int dl = l - lp;
      if (dl < 0) dl += Nt;
      s_row[(jr - 1) * Nt + lp] += c_tt * T.d2t[dl] + c_t * T.d1t[dl];
    }
  }
  wave_sync();
  if (lane == 0) s_row[q] += cc;
  wave_sync();
  double mx = 0.0;
  for (int col = lane; col < n; col += kWave) mx = fmax(mx, fabs(s_row[col]));
  mx = wave_max(mx);
  const double scale = 1.0 / mx;
  double* row = A + (int64_t)ci * stride + (int64_t)q * ld;
  if (lane == 0) rowscale[(int64_t)ci * n + q] = scale;
  for (int col = 2 * lane; col < n; col += 2 * kWave) {     // n is even
    double2 v;
    v.x = scale * s_row[col];
    v.y = scale * s_row[col + 1];
    *reinterpret_cast<double2*>(row + col) = v;
  }
  if (mixed) {
    for (int j = lane; j < M; j += kWave) {
      double v = 0.0;
      for (int lp = 0; lp < Nt; ++lp) v += s_ring[lp] * T.H[(int64_t)lp * M + j];
      row[n + j] = scale * v;
    }
  } else {
    // the ring holds two entries, at l and l + half: the same two products,
    // in the same order, as the dense sum
    const int lh = (l + half) % Nt;
    const int a = min(l, lh), b = max(l, lh);
    const double ra = s_ring[a], rb = s_ring[b];
    for (int j = lane; j < M; j += kWave) {
      double v = ra * T.H[(int64_t)a * M + j];
      v += rb * T.H[(int64_t)b * M + j];
      row[n + j] = scale * v;
    }
  }
  if (lane == 0) row[n + M] = -scale * ff;
  for (int col = n + M + 1 + lane; col < ld; col += kWave) row[col] = 0.0;
}

void launch_colloc_build(const BucketTables& T, const ChunkDesc& C, const NodeSamples& S,
                         double* A, int64_t mat_stride, double* rowscale, hipStream_t st) {
  dim3 grid((T.n + kBuildWaves - 1) / kBuildWaves, C.count);
  size_t shm = sizeof(double) * kBuildWaves * (size_t)(T.n + T.Nt);
  (void)hipFuncSetAttribute((const void*)colloc_build_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shm);
  hipLaunchKernelGGL(colloc_build_kernel, grid, dim3(64 * kBuildWaves), shm, st, T, C, S, A, mat_stride,
                     rowscale);
}

// ------------------------------------------- K4: knot evaluation and scatter

// One workgroup per floating circle.  For each assigned knot (rho*, phi*), the
// interpolation weights over the full diameter grid are barycentric Lagrange
// weights in rho times Ntheta-point periodic cardinals in theta; folded onto
// the unknowns they give e (interior) and eps (ring):
//   C[i, Xi_m] = e^T W[:, :M] - eps^T H,   r_i = e^T W[:, M],   C_ii = 1.
// Knots go in chunks of 32; for each chunk [E | -eps] [W ; H] is a
// (32 x (n + Ntheta)) ((n + Ntheta) x (M+1)) product (H zero in column M):
// E and -eps are formed in LDS 32 columns at a time from the radial and
// angular weights, the rows of W and H are staged beside them, and the four
// wavefronts accumulate the product on MFMA (wavefront w: knots
// 16 (w mod 2) .., every other 16-column block).
namespace {
constexpr int kEK = 32;           // knots per chunk
constexpr int kEQ = 32;           // interior nodes per staged block
constexpr int kEMaxCB = 5;        // column blocks per wavefront: nrhs <= 160
constexpr int kEThreads = 256;
}

__global__ __launch_bounds__(kEThreads) __attribute__((amdgpu_waves_per_eu(2))) void eval_scatter_kernel(BucketTables T, ChunkDesc C,
                                                                 const double* __restrict__ A0,
                                                                 int64_t stride, double* __restrict__ val,
                                                                 double* __restrict__ bvec) {
  extern __shared__ double sh[];
  const int Nc1 = T.Nc + 1, Nt = T.Nt, n = T.n, M = T.M, nrhs = T.nrhs, ld = T.ld;
  const int NCB = (nrhs + 15) / 16, NC = NCB * 16;
  const int sx = Nc1 | 1, st = Nt | 1;               // odd strides
  double* lx = sh;                                    // [kEK][sx]
  double* lt = lx + kEK * sx;                         // [kEK][st]
  double* eps = lt + kEK * st;                        // [kEK][st]
  double* Eb = eps + kEK * st;                        // [kEK][kEQ + 1]
  double* Wb = Eb + kEK * (kEQ + 1);                  // [kEQ][NC + 1]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int rb = w & 1, cb0 = w >> 1;                 // row block, first column block
  const int ci = blockIdx.x;
  const int f = C.fl[ci];
  const int m = C.float_ids[f];
  const double* A = A0 + (int64_t)ci * stride;
  const int64_t klo = C.fk_off[f], khi = C.fk_off[f + 1];
  const double cxm = C.cx[m], cym = C.cy[m], rm = C.rad[m];
  const int half = Nt / 2;
  typedef double dbl4 __attribute__((ext_vector_type(4)));
  for (int64_t base = klo; base < khi; base += kEK) {
    const int cnt = (int)min<int64_t>(kEK, khi - base);
    // radial weights (one thread per knot) ...
    if (tid < kEK) {
      const int t = tid;
      if (t < cnt) {
        const int i = C.fk_ids[base + t];
        const double dx = C.kx[i] - cxm, dy = C.ky[i] - cym;
        const double rho = sqrt(dx * dx + dy * dy) / rm;
        int exact = -1;
        double ssum = 0.0;
        for (int j = 0; j < Nc1; ++j) {
          const double d = rho - T.xr[j];
          if (d == 0.0) exact = j;
          else ssum += T.bw[j] / d;
        }
        for (int j = 0; j < Nc1; ++j)
          lx[t * sx + j] = (exact >= 0) ? (j == exact ? 1.0 : 0.0) : (T.bw[j] / (rho - T.xr[j])) / ssum;
      } else {
        for (int j = 0; j < Nc1; ++j) lx[t * sx + j] = 0.0;
      }
    }
    // ... and angular cardinals (all threads)
    const double hstep = kTwoPiD / Nt;
    for (int idx = tid; idx < kEK * Nt; idx += kEThreads) {
      const int t = idx / Nt, l = idx - t * Nt;
      double v = 0.0;
      if (t < cnt) {
        const int i = C.fk_ids[base + t];
        const double phi = atan2(C.ky[i] - cym, C.kx[i] - cxm);
        // the cardinal is 2 pi-periodic in the angle difference: reduce it to
        // [-pi, pi] first, so that Nt x stays small wherever sin(x) is (else a
        // knot at angle -pi next to the node at +pi loses all digits)
        double d = phi - hstep * l;
        d -= kTwoPiD * rint(d / kTwoPiD);
        const double x = 0.5 * d;
        double sxx, cxx;
        sincos(x, &sxx, &cxx);
        // periodic cardinal sin(Nt x) cos(x) / (Nt sin(x)) at half-angle x
        v = (fabs(sxx) < 1e-15) ? 1.0 : sin(Nt * x) * cxx / (Nt * sxx);
      }
      lt[t * st + l] = v;
    }
    __syncthreads();
    // ring weights eps[t][l]
    for (int idx = tid; idx < kEK * Nt; idx += kEThreads) {
      const int t = idx / Nt, l = idx - t * Nt;
      int lq = l + half;
      if (lq >= Nt) lq -= Nt;
      eps[t * st + l] = lx[t * sx] * lt[t * st + l] + lx[t * sx + Nc1 - 1] * lt[t * st + lq];
    }
    dbl4 acc[kEMaxCB];
#pragma unroll
    for (int u = 0; u < kEMaxCB; ++u) acc[u] = dbl4{0.0, 0.0, 0.0, 0.0};
    auto mma = [&]() {
#pragma unroll
      for (int ks = 0; ks < kEQ / 4; ++ks) {
        const double a = Eb[(16 * rb + li) * (kEQ + 1) + 4 * ks + lk];
#pragma unroll
        for (int u = 0; u < kEMaxCB; ++u) {
          const int cb = cb0 + 2 * u;
          if (cb < NCB) {
            const double bb = Wb[(4 * ks + lk) * (NC + 1) + 16 * cb + li];
            acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc[u], 0, 0, 0);
          }
        }
      }
    };
    for (int q0 = 0; q0 < n; q0 += kEQ) {
      const int qn = min(kEQ, n - q0);
      // E block: e_t(q) = lx[t][k] lt[t][l'] + lx[t][Nc - k] lt[t][l' + Nt/2]
      for (int idx = tid; idx < kEK * kEQ; idx += kEThreads) {
        const int t = idx / kEQ, qq = idx - t * kEQ;
        double e = 0.0;
        if (qq < qn) {
          const int q = q0 + qq;
          const int k = q / Nt + 1;
          const int lp = q - (k - 1) * Nt;
          int lq = lp + half;
          if (lq >= Nt) lq -= Nt;
          e = lx[t * sx + k] * lt[t * st + lp] + lx[t * sx + (Nc1 - 1 - k)] * lt[t * st + lq];
        }
        Eb[t * (kEQ + 1) + qq] = e;
      }
      // W rows q0 .. q0 + qn (columns n .. n + nrhs), zero-padded: every load
      // of the block issued before the first LDS store (entries outside it
      // read the valid A[0] and are zeroed on the way in)
      {
        constexpr int kWPT = 8;                 // loads in flight per thread and pass
#pragma unroll 1
        for (int i0 = 0; i0 < kEQ * NC; i0 += kWPT * kEThreads) {
          double wv[kWPT];
#pragma unroll
          for (int k = 0; k < kWPT; ++k) {
            const int idx = i0 + tid + kEThreads * k, qq = idx / NC, c = idx - qq * NC;
            const bool ok = idx < kEQ * NC && qq < qn && c < nrhs;
            wv[k] = A[ok ? (int64_t)(q0 + qq) * ld + n + c : 0];
          }
#pragma unroll
          for (int k = 0; k < kWPT; ++k) {
            const int idx = i0 + tid + kEThreads * k, qq = idx / NC, c = idx - qq * NC;
            if (idx < kEQ * NC) Wb[qq * (NC + 1) + c] = (qq < qn && c < nrhs) ? wv[k] : 0.0;
          }
        }
      }
      __syncthreads();
      mma();
      __syncthreads();
    }
    // the boundary-ring correction -eps H of the knot columns (c < M) as more
    // blocks of the same product: E block -eps[t][l], W block H[l][c]
    for (int l0 = 0; l0 < Nt; l0 += kEQ) {
      const int ln = min(kEQ, Nt - l0);
      for (int idx = tid; idx < kEK * kEQ; idx += kEThreads) {
        const int t = idx / kEQ, qq = idx - t * kEQ;
        Eb[t * (kEQ + 1) + qq] = qq < ln ? -eps[t * st + l0 + qq] : 0.0;
      }
      {
        constexpr int kWPT = 8;
#pragma unroll 1
        for (int i0 = 0; i0 < kEQ * NC; i0 += kWPT * kEThreads) {
          double hv[kWPT];
#pragma unroll
          for (int k = 0; k < kWPT; ++k) {
            const int idx = i0 + tid + kEThreads * k, qq = idx / NC, c = idx - qq * NC;
            const bool ok = idx < kEQ * NC && qq < ln && c < M;
            hv[k] = T.H[ok ? (int64_t)(l0 + qq) * M + c : 0];
          }
#pragma unroll
          for (int k = 0; k < kWPT; ++k) {
            const int idx = i0 + tid + kEThreads * k, qq = idx / NC, c = idx - qq * NC;
            if (idx < kEQ * NC) Wb[qq * (NC + 1) + c] = (qq < ln && c < M) ? hv[k] : 0.0;
          }
        }
      }
      __syncthreads();
      mma();
      __syncthreads();
    }
    // D layout: acc[u][v] is knot 16 rb + 4 v + lk, column 16 cb + li.  The
    // four knots' rows are looked up once, all loads at once (inside the
    // store loop every lookup would wait for the one before: the stores
    // may alias the index arrays as far as the compiler knows)
    int kn[4];
    int64_t kro[4];
    {
      const int64_t lo = C.knot_off[m];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int t = 16 * rb + 4 * v + lk;
        kn[v] = C.fk_ids[base + (t < cnt ? t : 0)];
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) kro[v] = C.rowptr[kn[v]] + ((kn[v] < lo) ? 1 : 0);
    }
#pragma unroll
    for (int u = 0; u < kEMaxCB; ++u) {
      const int cb = cb0 + 2 * u;
      const int c = 16 * cb + li;
      if (cb < NCB && c < nrhs) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int t = 16 * rb + 4 * v + lk;
          if (t < cnt) {
            const double x = acc[u][v];
            if (c < M) val[kro[v] + c] = x;
            else bvec[kn[v]] = x;
          }
        }
      }
    }
    if (tid < cnt) {
      const int i = C.fk_ids[base + tid];
      const int64_t lo = C.knot_off[m];
      val[C.rowptr[i] + ((i < lo) ? 0 : M)] = 1.0;
    }
    __syncthreads();
  }
}

void launch_eval_scatter(const BucketTables& T, const ChunkDesc& C, const double* A,
                         int64_t mat_stride, double* val, double* b, hipStream_t st) {
  const int NC = (T.nrhs + 15) / 16 * 16;
  const size_t shm = sizeof(double) * ((size_t)kEK * ((T.Nc + 1) | 1) + 2 * (size_t)kEK * (T.Nt | 1) +
                                       (size_t)kEK * (kEQ + 1) + (size_t)kEQ * (NC + 1));
  (void)hipFuncSetAttribute((const void*)eval_scatter_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shm);
  hipLaunchKernelGGL(eval_scatter_kernel, dim3(C.count), dim3(kEThreads), shm, st, T, C, A, mat_stride,
                     val, b);
}

}  // namespace pdd
