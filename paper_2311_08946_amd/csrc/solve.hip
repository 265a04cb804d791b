// Solve of the interfacial system C u = r (and C^T lambda = g for the
// adjoint) by BiCGStab on the device.  The paper solves C u = r with GMRES and
// a one-level restricted additive Schwarz preconditioner (Section 4, eqs.
// 42-45); C has a unit diagonal, and plain BiCGStab converges in hundreds of
// iterations on the covers here.
//
// Operator layout.  With one subdomain per row (eqs. 28-30, Section 3.2), row
// i of C holds C_ii and the entries of one circle's stencil, a contiguous
// range of knots (eq. 9); and the knots of circle m appear only in the rows
// assigned to m.  On the first solve of a system the values are re-laid out
// per row -- the stencil entries in knot order at rowptr[i] - i, the diagonal
// apart -- so that a product reads 8 bytes per entry and no column indices:
//   C x   : a wavefront per circle m, y_i = C_ii x_i + sum_j V_ij x_{s0 + j}
//           for the rows i assigned to m: the inputs at m's knots stay in
//           registers (x_{s0 + j} in lane j, read once per circle rather than
//           once per row), each row's entries one coalesced load (16 rows'
//           loads in flight), and a butterfly over the lanes adds 16 rows at
//           once; the boundary rows (C_ii alone) follow as one more list;
//   C^T x : a wavefront per circle m, its lanes over the knots j of m,
//           y_j = C_jj x_j + sum_{rows i of m} V_ij x_i, each row's entries
//           one coalesced load (16 rows' loads in flight) and x_i broadcast
//           from the lane that loaded it -- no atomics and no transposed copy.
// Rows of the averaged rule (eqs. 38-39) hold several stencils; those systems
// keep the CSR form (and a transposed CSR copy for C^T).
//
// One iteration is four launches: p = r + beta (p - omega v); v = A p with
// per-workgroup partial sums of (r0, v); t = A s with partial sums of (t, s),
// (t, t), where s = r - alpha v is formed from r and v wherever it is read
// and never stored; the x and r updates with partial sums of (r, r) and
// (r0, r).  Every kernel runs on a fixed grid of kGrid
// workgroups striding over its rows or circles, and each workgroup first adds
// the kGrid partial sums of the kernel before it -- every workgroup the same
// partials in the same fixed order, so all derive the same scalars (alpha,
// omega, beta, the stopping test) and results are bitwise reproducible
// without a separate reduction launch; workgroup 0 records them.  Every kernel
// returns at once after the stopping test has fired, which lets the host
// enqueue several iterations per status read; a one-workgroup status kernel
// per batch adds the last partials for the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "runtime.h"

namespace pdd {

namespace {

constexpr int kThreads = 256;        // every kernel: four wavefronts
constexpr int kGrid = 2048;          // workgroups of every iteration kernel (strided)
constexpr int kLanes = 16;           // lanes per row in the row products
constexpr int kRowsPerPass = kThreads / kLanes;
constexpr int kItersPerSync = 8;

enum { OP_CSR = 0, OP_ROWS_BY_CIRCLE = 1, OP_CIRCLES = 2 };

enum {
  S_RHO = 0, S_ALPHA, S_OMEGA, S_BETA, S_RV, S_TS, S_TT, S_RR, S_BB, S_TOL2, S_DONE, S_FAIL,
  S_ITER, S_RHO_PREV, S_COUNT
};

struct SolveCtx {
  // the operator A (C or C^T)
  int kind;
  const int64_t* rowptr;   // CSR row pointers of A (OP_CSR) or of C (blocked kinds)
  const int32_t* cols;     // OP_CSR
  const double* val;       // OP_CSR
  const double* vblk;      // blocked: stencil entries of row i at rowptr[i] - i
  const double* dg;        // blocked: diagonal
  const int64_t* knot_off; // blocked: knots of circle m are [knot_off[m], knot_off[m + 1])
  const int64_t* circ_off; // blocked: rows of circle m are circ_rows[circ_off[m] ..), m <= nc
                           // (list nc: the boundary rows)
  const int32_t* circ_rows;
  const int64_t* circ_roff; // blocked: rowptr[i] - i of the row at each circ_rows slot
  int32_t nc;
  int64_t N;
  double* x;
  double* r;
  double* r0;
  double* p;
  double* v;
  double* t;
  double* part_i;      // [2][kGrid] init: (b, b), (r, r)
  double* part_v;      // [kGrid]    spmv_v: (r0, v)
  double* part_t;      // [2][kGrid] spmv_t: (t, s), (t, t)
  double* part_x;      // [2][kGrid] update_xr: (r, r), (r0, r)
  double* sc;          // scalars, written by workgroup 0 of the kernel that derives them
  double* status;      // the host's record: the state after the last finished iteration
};

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Workgroup sum in a fixed order (wave sums, then the wave totals in order).
__device__ __forceinline__ double block_sum(double v, double* s) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) s[w] = v;
  __syncthreads();
  return s[0] + s[1] + s[2] + s[3];
}

// Sum of part[0:kGrid) in a fixed order (the same in every workgroup).
__device__ __forceinline__ double sum_parts(const double* __restrict__ part, double* s) {
  double a = 0.0;
#pragma unroll
  for (int i = 0; i < kGrid / kThreads; ++i) a += part[threadIdx.x + kThreads * i];
  return block_sum(a, s);
}

// The input vector of a product: y (ALPHA = false) or y - alpha z.
template <bool ALPHA>
struct In {
  static constexpr bool kTwoLoads = ALPHA;
  const double* y;
  const double* z;
  double alpha;
  __device__ __forceinline__ double operator()(int64_t j) const { return ALPHA ? y[j] - alpha * z[j] : y[j]; }
};

// Lane l's value, read by every lane (l wavefront-uniform).
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ int64_t readlane_i64(int64_t v, int l) {
  const int lo = __builtin_amdgcn_readlane((int)v, l), hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return ((int64_t)hi << 32) | (unsigned)lo;
}

// Sums of 16 rows held across a wavefront: p[u] is this lane's term of row
// u.  Four halving exchanges (lanes 32, 16, 8, 4 apart) each keep the half of
// the rows named by that lane bit and add the partner's terms of them, then
// two exchanges add the last four lanes: lanes 4u .. 4u + 3 end with the sum
// of row u (the same order of additions whichever of them holds it).
__device__ __forceinline__ double rows_sum16(const double (&p)[16], int lane) {
  double a8[8], a4[4], a2[2];
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
#pragma unroll
  for (int k = 0; k < 8; ++k) a8[k] = (b5 ? p[k + 8] : p[k]) + __shfl_xor(b5 ? p[k] : p[k + 8], 32, 64);
#pragma unroll
  for (int k = 0; k < 4; ++k) a4[k] = (b4 ? a8[k + 4] : a8[k]) + __shfl_xor(b4 ? a8[k] : a8[k + 4], 16, 64);
#pragma unroll
  for (int k = 0; k < 2; ++k) a2[k] = (b3 ? a4[k + 2] : a4[k]) + __shfl_xor(b3 ? a4[k] : a4[k + 2], 8, 64);
  double a = (b2 ? a2[1] : a2[0]) + __shfl_xor(b2 ? a2[0] : a2[1], 4, 64);
  a += __shfl_xor(a, 1, 64);
  return a + __shfl_xor(a, 2, 64);
}

// Visits every output (A x)_i once, in a partition fixed by the grid, calling
// sink(i, value) from one lane per output.
template <int OPK, class X, class Sink>
__device__ __forceinline__ void apply_op(const SolveCtx& c, const X& in, Sink& sink) {
  const int tid = threadIdx.x;
  if (OPK == OP_ROWS_BY_CIRCLE) {
    // C x by the circles the rows are assigned to: circle m's inputs x_j
    // (its knots, the stencil of each of its rows) stay in registers, x_{s0+j}
    // in lane j; its rows go sixteen at a time, lane j loading entry j of
    // each (a row per coalesced load) times its x_j, and rows_sum16 adds
    // them.  The boundary rows (C_ii alone) are the list after the last
    // circle's rows, spread over every thread.
    const int lane = tid & 63, u_out = (lane >> 2) & 15;
    for (int m = blockIdx.x * (kThreads / 64) + (tid >> 6); m < c.nc; m += gridDim.x * (kThreads / 64)) {
      const int64_t s0 = c.knot_off[m], len = c.knot_off[m + 1] - s0;
      const int64_t q0 = c.circ_off[m], q1 = c.circ_off[m + 1];
      if (q0 == q1) continue;
      const double x0 = lane < len ? in(s0 + lane) : 0.0;
      for (int64_t qb = q0; qb < q1; qb += 64) {
        const int cnt = (int)min((int64_t)64, q1 - qb);
        int64_t off = 0;
        int32_t row = 0;
        double dterm = 0.0;
        if (lane < cnt) {
          off = c.circ_roff[qb + lane];
          row = c.circ_rows[qb + lane];
          dterm = c.dg[row] * in(row);
        }
        for (int q = 0; q < cnt; q += 16) {
          // (the address is clamped and the value masked, so that every
          // load of the sixteen rows is in flight at once)
          double p[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int64_t o = readlane_i64(off, q + u);
            const bool okv = lane < len && q + u < cnt;
            const double v = c.vblk[okv ? o + lane : 0];
            p[u] = okv ? v * x0 : 0.0;
          }
          for (int64_t jb = 64; jb < len; jb += 64) {   // stencils of more than 64 knots
            const bool okj = jb + lane < len;
            const double xj = okj ? in(s0 + jb + lane) : 0.0;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
              const int64_t o = readlane_i64(off, q + u);
              const bool okv = okj && q + u < cnt;
              const double v = c.vblk[okv ? o + jb + lane : 0];
              p[u] += okv ? v * xj : 0.0;
            }
          }
          const double sum = rows_sum16(p, lane);
          const int src = q + u_out;
          const int32_t ri = __shfl(row, src, 64);
          const double dt = __shfl(dterm, src, 64);
          if ((lane & 3) == 0 && src < cnt) sink(ri, dt + sum);
        }
      }
    }
    for (int64_t q = c.circ_off[c.nc] + (int64_t)blockIdx.x * kThreads + tid; q < c.circ_off[c.nc + 1];
         q += (int64_t)gridDim.x * kThreads) {
      const int64_t i = c.circ_rows[q];
      sink(i, c.dg[i] * in(i));
    }
    return;
  }
  if (OPK == OP_CIRCLES) {
    // circle m: lanes over its knots j; its rows' offsets and inputs are
    // staged one per lane (64 rows at a time) and broadcast by readlane, so
    // the loop issues only the coalesced loads of the rows' entries, sixteen
    // rows' loads at a time
    const int lane = tid & 63;
    for (int m = blockIdx.x * (kThreads / 64) + (tid >> 6); m < c.nc; m += gridDim.x * (kThreads / 64)) {
      const int64_t s0 = c.knot_off[m], s1 = c.knot_off[m + 1];
      const int64_t q0 = c.circ_off[m], q1 = c.circ_off[m + 1];
      for (int64_t jb = s0; jb < s1; jb += 64) {
        const int64_t j = jb + lane;
        const bool ok = j < s1;
        double a0 = 0.0, a1 = 0.0;
        for (int64_t qb = q0; qb < q1; qb += 64) {
          const int cnt = (int)min((int64_t)64, q1 - qb);
          int64_t off = 0;
          double xi = 0.0;
          if (lane < cnt) {
            off = c.circ_roff[qb + lane] + (jb - s0);   // the row's entries of this chunk of knots
            xi = in(c.circ_rows[qb + lane]);
          }
          int q = 0;
          for (; q + 16 <= cnt; q += 16) {
            double v[16], x[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
              const int64_t o = readlane_i64(off, q + u);
              x[u] = readlane_f64(xi, q + u);
              v[u] = ok ? c.vblk[o + lane] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 16; u += 2) {
              a0 += v[u] * x[u];
              a1 += v[u + 1] * x[u + 1];
            }
          }
          for (; q + 4 <= cnt; q += 4) {
            double v[4], x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int64_t o = readlane_i64(off, q + u);
              x[u] = readlane_f64(xi, q + u);
              v[u] = ok ? c.vblk[o + lane] : 0.0;
            }
            a0 += v[0] * x[0];
            a1 += v[1] * x[1];
            a0 += v[2] * x[2];
            a1 += v[3] * x[3];
          }
          for (; q < cnt; ++q) {
            const int64_t o = readlane_i64(off, q);
            const double x = readlane_f64(xi, q);
            if (ok) a0 += c.vblk[o + lane] * x;
          }
        }
        if (ok) sink(j, c.dg[j] * in(j) + (a0 + a1));
      }
    }
    return;
  }
  const int sub = tid & (kLanes - 1);
  for (int64_t base = (int64_t)blockIdx.x * kRowsPerPass; base < c.N; base += (int64_t)gridDim.x * kRowsPerPass) {
    const int64_t i = base + tid / kLanes;
    double acc = 0.0;
    if (i < c.N) {                           // uniform within the row's lanes
      const int64_t lo = c.rowptr[i], hi = c.rowptr[i + 1];
      for (int64_t k = lo + sub; k < hi; k += kLanes) acc += c.val[k] * in(c.cols[k]);
    }
    for (int off = kLanes / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kLanes);
    if (sub == 0 && i < c.N) sink(i, acc);
  }
}

// x-independent start: r = b - A x (x = 0 unless a guess is given, whose
// product the caller left in t), partial sums of (b, b) and (r, r).
__global__ __launch_bounds__(kThreads) void init_kernel(SolveCtx c, const double* __restrict__ b, int use_guess) {
  __shared__ double s4[4];
  double pbb = 0.0, prr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < c.N; i += (int64_t)gridDim.x * kThreads) {
    const double ri = b[i] - (use_guess ? c.t[i] : 0.0);
    if (!use_guess) c.x[i] = 0.0;
    c.r[i] = ri;
    c.r0[i] = ri;
    c.p[i] = 0.0;
    c.v[i] = 0.0;
    pbb += b[i] * b[i];
    prr += ri * ri;
  }
  const double sbb = block_sum(pbb, s4);
  const double srr = block_sum(prr, s4);
  if (threadIdx.x == 0) {
    c.part_i[blockIdx.x] = sbb;
    c.part_i[kGrid + blockIdx.x] = srr;
  }
}

// t = A x (the product of a starting guess).
template <int OPK>
__global__ __launch_bounds__(kThreads) void guess_product_kernel(SolveCtx c) {
  struct Sink {
    const SolveCtx& c;
    __device__ void operator()(int64_t i, double y) { c.t[i] = y; }
  } sink{c};
  apply_op<OPK>(c, In<false>{c.x, nullptr, 0.0}, sink);
}

// The scalars after an x, r update (or after init when FIRST): the stopping
// test and beta.  Run by every thread of every workgroup of the caller on the
// same partials; returns true if the iteration goes on.  REC: record them
// (workgroup 0 of update_p writes sc; the status kernel writes the host's
// record and leaves sc alone).
struct Next {
  double rr, rho, beta, bb, tol2, iter;
  bool done, fail;
};

__device__ Next next_state(const SolveCtx& c, bool first, double rtol, double* s) {
  const double* sc = c.sc;
  Next z{};
  if (first) {
    z.bb = sum_parts(c.part_i, s);
    z.rr = sum_parts(c.part_i + kGrid, s);
    z.rho = z.rr;                    // (r0, r) with r0 = r
    z.beta = 0.0;
    z.tol2 = rtol * rtol * z.bb;
    z.iter = 0.0;
    z.done = z.rr <= z.tol2;
    z.fail = false;
    return z;
  }
  z.rr = sum_parts(c.part_x, s);
  z.rho = sum_parts(c.part_x + kGrid, s);
  z.bb = sc[S_BB];
  z.tol2 = sc[S_TOL2];
  z.beta = (z.rho / sc[S_RHO_PREV]) * (sc[S_ALPHA] / sc[S_OMEGA]);
  z.iter = sc[S_ITER] + 1.0;
  const bool bad = !(z.rr == z.rr) || !isfinite(z.beta) || sc[S_OMEGA] == 0.0 || z.rho == 0.0;
  z.done = z.rr <= z.tol2 || bad;
  z.fail = !(z.rr <= z.tol2) && bad;
  return z;
}

__device__ void record(double* rec, const Next& z, bool first) {
  rec[S_RR] = z.rr;
  rec[S_ITER] = z.iter;
  rec[S_DONE] = z.done ? 1.0 : 0.0;
  rec[S_FAIL] = z.fail ? 1.0 : 0.0;
  if (first) {
    rec[S_BB] = z.bb;
    rec[S_TOL2] = z.tol2;
    rec[S_ALPHA] = 1.0;
    rec[S_OMEGA] = 1.0;
  }
  if (!z.done) {
    rec[S_RHO] = z.rho;
    rec[S_BETA] = z.beta;
  }
}

// p = r + beta (p - omega v), after the scalars of the previous x, r update.
__global__ __launch_bounds__(kThreads) void update_p_kernel(SolveCtx c, int first, double rtol) {
  __shared__ double s4[4];
  __shared__ int stop;
  // workgroup 0 may set S_DONE while others start: read it once per workgroup
  if (threadIdx.x == 0) stop = (!first && c.sc[S_DONE] != 0.0) ? 1 : 0;
  __syncthreads();
  if (stop) return;
  const Next z = next_state(c, first != 0, rtol, s4);
  if (blockIdx.x == 0 && threadIdx.x == 0) record(c.sc, z, first != 0);
  if (z.done) return;
  const double omega = first ? 1.0 : c.sc[S_OMEGA];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < c.N; i += (int64_t)gridDim.x * kThreads)
    c.p[i] = c.r[i] + z.beta * (c.p[i] - omega * c.v[i]);
}

// v = A p, partial sums of (r0, v)
template <int OPK>
__global__ __launch_bounds__(kThreads) void spmv_v_kernel(SolveCtx c) {
  __shared__ double s4[4];
  if (c.sc[S_DONE] != 0.0) return;
  struct Sink {
    const SolveCtx& c;
    double prv;
    __device__ void operator()(int64_t i, double y) {
      c.v[i] = y;
      prv += c.r0[i] * y;
    }
  } sink{c, 0.0};
  apply_op<OPK>(c, In<false>{c.p, nullptr, 0.0}, sink);
  const double sv = block_sum(sink.prv, s4);
  if (threadIdx.x == 0) c.part_v[blockIdx.x] = sv;
}

// alpha = rho / (r0, v) (every workgroup adds the partial sums of (r0, v)
// itself); t = A s with s = r - alpha v formed from r and v wherever it is
// read (s is never stored), partial sums of (t, s) and (t, t)
template <int OPK>
__global__ __launch_bounds__(kThreads) void spmv_t_kernel(SolveCtx c) {
  __shared__ double s4[4];
  if (c.sc[S_DONE] != 0.0) return;
  const double rv = sum_parts(c.part_v, s4);
  const double alpha = c.sc[S_RHO] / rv;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c.sc[S_RV] = rv;
    c.sc[S_ALPHA] = alpha;
  }
  struct Sink {
    const SolveCtx& c;
    double alpha, pts, ptt;
    __device__ void operator()(int64_t i, double y) {
      c.t[i] = y;
      pts += y * (c.r[i] - alpha * c.v[i]);
      ptt += y * y;
    }
  } sink{c, alpha, 0.0, 0.0};
  apply_op<OPK>(c, In<true>{c.r, c.v, alpha}, sink);
  const double sts = block_sum(sink.pts, s4);
  const double stt = block_sum(sink.ptt, s4);
  if (threadIdx.x == 0) {
    c.part_t[blockIdx.x] = sts;
    c.part_t[kGrid + blockIdx.x] = stt;
  }
}

// omega = (t, s) / (t, t); x += alpha p + omega s; r = s - omega t with
// s = r - alpha v; partial sums of (r, r) and (r0, r)
__global__ __launch_bounds__(kThreads) void update_xr_kernel(SolveCtx c) {
  __shared__ double s4[4];
  if (c.sc[S_DONE] != 0.0) return;
  const double ts = sum_parts(c.part_t, s4);
  const double tt = sum_parts(c.part_t + kGrid, s4);
  const double omega = (tt > 0.0) ? ts / tt : 0.0;
  const double alpha = c.sc[S_ALPHA];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c.sc[S_TS] = ts;
    c.sc[S_TT] = tt;
    c.sc[S_OMEGA] = omega;
    c.sc[S_RHO_PREV] = c.sc[S_RHO];    // update_p replaces S_RHO while its workgroups read this
  }
  double prr = 0.0, prho = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < c.N; i += (int64_t)gridDim.x * kThreads) {
    const double si = c.r[i] - alpha * c.v[i];
    c.x[i] = c.x[i] + alpha * c.p[i] + omega * si;
    const double ri = si - omega * c.t[i];
    c.r[i] = ri;
    prr += ri * ri;
    prho += c.r0[i] * ri;
  }
  const double srr = block_sum(prr, s4);
  const double srho = block_sum(prho, s4);
  if (threadIdx.x == 0) {
    c.part_x[blockIdx.x] = srr;
    c.part_x[kGrid + blockIdx.x] = srho;
  }
}

// The host's record after a batch: the state sc holds once stopped, else the
// one the next update_p would derive (sc is not touched).
__global__ __launch_bounds__(kThreads) void status_kernel(SolveCtx c, int first, double rtol) {
  __shared__ double s4[4];
  if (!first && c.sc[S_DONE] != 0.0) {
    if (threadIdx.x < S_COUNT) c.status[threadIdx.x] = c.sc[threadIdx.x];
    return;
  }
  const Next z = next_state(c, first != 0, rtol, s4);
  if (threadIdx.x == 0) {
    for (int k = 0; k < S_COUNT; ++k) c.status[k] = c.sc[k];
    record(c.status, z, first != 0);
  }
}

__global__ void gather_kernel(const int64_t* __restrict__ perm, const double* __restrict__ src,
                              double* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

// The circle-blocked values of C from its CSR: a 16-lane group per row puts
// C_ii into dg and the stencil entries at rowptr[i] - i + (column - so_i).
__global__ __launch_bounds__(kThreads) void form_blocked_kernel(const int64_t* __restrict__ rowptr,
                                                                const int32_t* __restrict__ cols,
                                                                const double* __restrict__ val,
                                                                const int32_t* __restrict__ so, int64_t N,
                                                                double* __restrict__ vblk, double* __restrict__ dg) {
  const int sub = threadIdx.x & (kLanes - 1);
  const int64_t i = (int64_t)blockIdx.x * kRowsPerPass + threadIdx.x / kLanes;
  if (i >= N) return;
  const int64_t lo = rowptr[i], hi = rowptr[i + 1];
  for (int64_t k = lo + sub; k < hi; k += kLanes) {
    const int32_t col = cols[k];
    if (col == i) dg[i] = val[k];
    else vblk[lo - i + (col - so[i])] = val[k];
  }
}

// Dense [A | b] of order np >= N for the operator A (C or C^T) in CSR,
// row-major with leading dimension ld, zeroed beforehand: a workgroup per
// row of A scatters its entries; padding rows get a unit diagonal; column np
// holds the right-hand side (zero on padding rows).
__global__ void dense_scatter_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ cols,
                                     const double* __restrict__ val, const double* __restrict__ b, int64_t N,
                                     int np, double* __restrict__ A, int ld) {
  const int64_t i = blockIdx.x;
  double* row = A + i * ld;
  if (i < N) {
    for (int64_t k = rowptr[i] + threadIdx.x; k < rowptr[i + 1]; k += blockDim.x) row[cols[k]] = val[k];
    if (threadIdx.x == 0) row[np] = b[i];
  } else if (threadIdx.x == 0) {
    row[i] = 1.0;
  }
}

// u = the solution column; |b - A u|^2 and |b|^2 into out[0], out[1], summed
// by one workgroup in a fixed order.
__global__ __launch_bounds__(kThreads) void dense_finish_kernel(
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ cols, const double* __restrict__ val,
    const double* __restrict__ b, int64_t N, int np, const double* __restrict__ A, int ld,
    double* __restrict__ u, double* __restrict__ out) {
  __shared__ double s4[4];
  double rr = 0.0, bb = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += kThreads) {
    u[i] = A[i * ld + np];
    double ax = 0.0;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) ax += val[k] * A[(int64_t)cols[k] * ld + np];
    const double ri = b[i] - ax;
    rr += ri * ri;
    bb += b[i] * b[i];
  }
  rr = block_sum(rr, s4);
  bb = block_sum(bb, s4);
  if (threadIdx.x == 0) {
    out[0] = rr;
    out[1] = bb;
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

// Circle-blocked structure of C on the device (see the top of this file),
// when every row holds its diagonal and one circle's stencil in column
// order; otherwise (rule AVERAGED) blocked_ok stays false.  Caller holds the
// cover's lock.
void ensure_blocked(pdd_cover cover) {
  DeviceCover& D = cover->D;
  if (D.have_blocked) return;
  const HostCover& H = cover->H;
  const int64_t N = H.N();
  bool ok = H.pairs == nullptr;
  std::vector<int32_t> so(N, 0);
  std::vector<int64_t> coff(H.nc + 2, 0);   // the boundary rows last, as list nc
  for (int64_t i = 0; ok && i < N; ++i) {
    const int64_t lo = H.rowptr[i], len = H.rowptr[i + 1] - lo;
    const int32_t m = H.assigned[i];
    if (m < 0) {                           // boundary row: C_ii alone
      ok = len == 1 && H.cols[lo] == i;
      ++coff[H.nc + 1];
      continue;
    }
    const int64_t s0 = H.knot_off[m], s1 = H.knot_off[m + 1];
    ok = len == s1 - s0 + 1 && (i < s0 || i >= s1);
    for (int64_t k = lo, j = s0; ok && k < lo + len; ++k) {
      if (H.cols[k] == i) continue;
      ok = H.cols[k] == j++;
    }
    so[i] = (int32_t)s0;
    ++coff[m + 1];
  }
  if (ok) {
    for (int32_t m = 0; m <= H.nc; ++m) coff[m + 1] += coff[m];
    std::vector<int32_t> rows(coff[H.nc + 1]);
    std::vector<int64_t> roff(coff[H.nc + 1]);
    std::vector<int64_t> fill(coff.begin(), coff.end() - 1);
    for (int64_t i = 0; i < N; ++i) {
      const int64_t q = fill[H.assigned[i] >= 0 ? H.assigned[i] : H.nc]++;
      rows[q] = (int32_t)i;
      roff[q] = H.rowptr[i] - i;
    }
    D.blk_so.upload(so);
    D.blk_circ_off.upload(coff);
    D.blk_circ_rows.upload(rows);
    D.blk_circ_roff.upload(roff);
  }
  D.blocked_ok = ok;
  D.have_blocked = true;
}

// The operator of a solve in the form its kernels read, formed on first use
// (the structure per cover, the values per system) and synchronised so that
// solves on other streams see it complete.  Blocked C serves both C and C^T;
// otherwise C^T needs its CSR pattern and values.
void prepare_operator(pdd_system sys, bool transpose, hipStream_t st) {
  std::lock_guard<std::mutex> lk(sys->cover->solve_mu);
  DeviceCover& D = sys->cover->D;
  const HostCover& H = sys->cover->H;
  const int64_t N = H.N(), nnz = H.rowptr.back();
  ensure_blocked(sys->cover);
  if (D.blocked_ok) {
    if (sys->have_vblk) return;
    sys->vblk.alloc(std::max<int64_t>(1, nnz - N) * sizeof(double));
    sys->dg.alloc(std::max<int64_t>(1, N) * sizeof(double));
    if (N > 0)
      hipLaunchKernelGGL(form_blocked_kernel, dim3((unsigned)((N + kRowsPerPass - 1) / kRowsPerPass)),
                         dim3(kThreads), 0, st, D.rowptr.ptr<int64_t>(), D.cols.ptr<int32_t>(),
                         sys->val.ptr<double>(), D.blk_so.ptr<int32_t>(), N, sys->vblk.ptr<double>(),
                         sys->dg.ptr<double>());
    PDD_HIP(hipGetLastError());
    PDD_HIP(hipStreamSynchronize(st));
    sys->have_vblk = true;
    return;
  }
  if (!transpose) return;
  ensure_transpose(sys->cover);
  if (sys->val_t.bytes() == 0) {     // C^T values, formed once per system
    sys->val_t.alloc(std::max<int64_t>(1, nnz) * sizeof(double));
    if (nnz > 0)
      hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st,
                         D.rt_perm.ptr<int64_t>(), sys->val.ptr<double>(), sys->val_t.ptr<double>(), nnz);
    PDD_HIP(hipGetLastError());
    PDD_HIP(hipStreamSynchronize(st));
  }
}

// Whether the form a solve needs exists already (the allocation-free entry
// point cannot form it).  Caller holds the cover's lock.
bool operator_ready(pdd_system sys, bool transpose) {
  const DeviceCover& D = sys->cover->D;
  if (!D.have_blocked) return false;
  if (D.blocked_ok) return sys->have_vblk;
  return !transpose || (D.have_transpose && sys->val_t.bytes() > 0);
}

namespace {

// Doubles of the BiCGStab work area for N unknowns: r, r0, p, v, t, the
// partial sums of the kernels, the scalars and the host's record.
int64_t work_doubles(int64_t N) { return 5 * N + 7 * (int64_t)kGrid + 2 * S_COUNT; }

// Points the context at the operator (prepared by prepare_operator) and
// carves the work area w (work_doubles(N) doubles) into its vectors.
void bind(SolveCtx& c, pdd_system sys, bool transpose, double* u, double* w) {
  const DeviceCover& D = sys->cover->D;
  const int64_t N = sys->cover->H.N();
  if (D.blocked_ok) {
    c.kind = transpose ? OP_CIRCLES : OP_ROWS_BY_CIRCLE;
    c.rowptr = D.rowptr.ptr<int64_t>();
    c.vblk = sys->vblk.ptr<double>();
    c.dg = sys->dg.ptr<double>();
    c.knot_off = D.knot_off.ptr<int64_t>();
    c.circ_off = D.blk_circ_off.ptr<int64_t>();
    c.circ_rows = D.blk_circ_rows.ptr<int32_t>();
    c.circ_roff = D.blk_circ_roff.ptr<int64_t>();
    c.nc = sys->cover->H.nc;
  } else {
    c.kind = OP_CSR;
    c.rowptr = transpose ? D.rt_rowptr.ptr<int64_t>() : D.rowptr.ptr<int64_t>();
    c.cols = transpose ? D.rt_cols.ptr<int32_t>() : D.cols.ptr<int32_t>();
    c.val = transpose ? sys->val_t.ptr<double>() : sys->val.ptr<double>();
  }
  c.N = N;
  c.x = u;
  c.r = w;
  c.r0 = c.r + N;
  c.p = c.r0 + N;
  c.v = c.p + N;
  c.t = c.v + N;
  c.part_i = c.t + N;
  c.part_v = c.part_i + 2 * kGrid;
  c.part_t = c.part_v + kGrid;
  c.part_x = c.part_t + 2 * kGrid;
  c.sc = c.part_x + 2 * kGrid;
  c.status = c.sc + S_COUNT;
}

template <int OPK>
void launch_iterations(const SolveCtx& c, hipStream_t st, int first, int count, double rtol) {
  for (int k = 0; k < count; ++k) {
    hipLaunchKernelGGL(update_p_kernel, dim3(kGrid), dim3(kThreads), 0, st, c, k == 0 ? first : 0, rtol);
    hipLaunchKernelGGL(spmv_v_kernel<OPK>, dim3(kGrid), dim3(kThreads), 0, st, c);
    hipLaunchKernelGGL(spmv_t_kernel<OPK>, dim3(kGrid), dim3(kThreads), 0, st, c);
    hipLaunchKernelGGL(update_xr_kernel, dim3(kGrid), dim3(kThreads), 0, st, c);
  }
}

// r = b - A x (x = 0, or the guess in x), r0 = r.
void launch_init(const SolveCtx& c, const double* b, bool guess, hipStream_t st) {
  if (guess) {
    if (c.kind == OP_CSR) hipLaunchKernelGGL(guess_product_kernel<OP_CSR>, dim3(kGrid), dim3(kThreads), 0, st, c);
    else if (c.kind == OP_ROWS_BY_CIRCLE)
      hipLaunchKernelGGL(guess_product_kernel<OP_ROWS_BY_CIRCLE>, dim3(kGrid), dim3(kThreads), 0, st, c);
    else hipLaunchKernelGGL(guess_product_kernel<OP_CIRCLES>, dim3(kGrid), dim3(kThreads), 0, st, c);
  }
  hipLaunchKernelGGL(init_kernel, dim3(kGrid), dim3(kThreads), 0, st, c, b, guess ? 1 : 0);
  PDD_HIP(hipGetLastError());
}

// Enqueues the next batch of at most kItersPerSync iterations after `enq`
// enqueued ones, then the status kernel that writes the host's record to
// c.status; returns the new count.
int enqueue_batch(const SolveCtx& c, hipStream_t st, int enq, int max_iter, double rtol) {
  const int batch = std::min(kItersPerSync, max_iter - enq);
  const int first = enq == 0 ? 1 : 0;
  if (c.kind == OP_CSR) launch_iterations<OP_CSR>(c, st, first, batch, rtol);
  else if (c.kind == OP_ROWS_BY_CIRCLE) launch_iterations<OP_ROWS_BY_CIRCLE>(c, st, first, batch, rtol);
  else launch_iterations<OP_CIRCLES>(c, st, first, batch, rtol);
  enq += batch;
  hipLaunchKernelGGL(status_kernel, dim3(1), dim3(kThreads), 0, st, c, enq == 0 ? 1 : 0, rtol);
  PDD_HIP(hipGetLastError());
  return enq;
}

struct SolveParams {
  double rtol;
  int max_iter;
  bool guess;
  int method;
};

SolveParams params(const pdd_solve_opts* opts) {
  return {(opts && opts->rtol > 0.0) ? opts->rtol : 1e-12,
          (opts && opts->max_iter > 0) ? opts->max_iter : 2000, opts && opts->use_guess,
          opts ? opts->method : PDD_SOLVE_BICGSTAB};
}

constexpr int64_t kDirectMax = 4096;   // largest order of the batched LU's panel classes

// PDD_SOLVE_DIRECT_SMALL: [A | b] (A = C or C^T) formed densely and solved by
// the batched LU with partial pivoting (one matrix, one right-hand side,
// eliminated and back-substituted inside the factorisation); reports the
// relative residual |b - A u| / |b|.
pdd_status direct_impl(pdd_system sys, const double* b, double* u, bool transpose, hipStream_t st,
                       pdd_solve_info* info) {
  const DeviceCover& D = sys->cover->D;
  const int64_t N = sys->cover->H.N();
  if (N > kDirectMax)
    return fail(PDD_EINVAL, "pdd_solve_G: the direct method takes at most " + std::to_string(kDirectMax) +
                                " knots, the system has " + std::to_string(N));
  if (N == 0) {
    if (info) *info = pdd_solve_info{0, 1, 0.0};
    return PDD_OK;
  }
  if (transpose) {                   // the CSR of C^T (small: N <= 4096)
    std::lock_guard<std::mutex> lk(sys->cover->solve_mu);
    ensure_transpose(sys->cover);
    const int64_t nnz = sys->cover->H.rowptr.back();
    if (sys->val_t.bytes() == 0) {
      sys->val_t.alloc(std::max<int64_t>(1, nnz) * sizeof(double));
      hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st,
                         D.rt_perm.ptr<int64_t>(), sys->val.ptr<double>(), sys->val_t.ptr<double>(), nnz);
      PDD_HIP(hipGetLastError());
      PDD_HIP(hipStreamSynchronize(st));
    }
  }
  const int64_t* rowptr = transpose ? D.rt_rowptr.ptr<int64_t>() : D.rowptr.ptr<int64_t>();
  const int32_t* cols = transpose ? D.rt_cols.ptr<int32_t>() : D.cols.ptr<int32_t>();
  const double* val = transpose ? sys->val_t.ptr<double>() : sys->val.ptr<double>();
  const int np = (int)((N + 31) / 32 * 32);
  const int ld = np + 16;
  DevBuf mat, piv, status, work, out;
  mat.alloc((size_t)np * ld * sizeof(double));
  piv.alloc((size_t)np * sizeof(int32_t));
  status.alloc(sizeof(int32_t));
  work.alloc(lu_work_bytes_per_matrix(np));
  out.alloc(2 * sizeof(double));
  PDD_HIP(hipMemsetAsync(mat.ptr<void>(), 0, mat.bytes(), st));
  PDD_HIP(hipMemsetAsync(status.ptr<void>(), 0, sizeof(int32_t), st));
  hipLaunchKernelGGL(dense_scatter_kernel, dim3((unsigned)np), dim3(64), 0, st, rowptr, cols, val, b, N, np,
                     mat.ptr<double>(), ld);
  PDD_HIP(hipGetLastError());
  LuItem it{};
  it.A = mat.ptr<double>();
  it.piv = piv.ptr<int32_t>();
  it.status = status.ptr<int32_t>();
  it.work = work.ptr<LuWork>();
  it.uinv = reinterpret_cast<double*>(work.ptr<char>() + lu_work_header_bytes());
  it.n = np;
  it.ld = ld;
  it.nrhs = 1;
  it.cls = lu_panel_class(np);
  int32_t stat = 0;
  double host[2] = {0.0, 0.0};
  {
    LuPlan plan;
    plan.build(std::vector<LuItem>{it});
    plan.launch(st, 1 << 30);
    hipLaunchKernelGGL(dense_finish_kernel, dim3(1), dim3(kThreads), 0, st, rowptr, cols, val, b, N, np,
                       mat.ptr<double>(), ld, u, out.ptr<double>());
    PDD_HIP(hipGetLastError());
    PDD_HIP(hipMemcpyAsync(host, out.ptr<void>(), sizeof host, hipMemcpyDeviceToHost, st));
    PDD_HIP(hipMemcpyAsync(&stat, status.ptr<void>(), sizeof stat, hipMemcpyDeviceToHost, st));
    PDD_HIP(hipStreamSynchronize(st));   // the plan and the buffers are released on return
  }
  const double rel = host[1] > 0.0 ? std::sqrt(host[0] / host[1]) : 0.0;
  if (info) *info = pdd_solve_info{1, stat ? 0 : 1, rel};
  if (stat) return fail(PDD_EBREAKDOWN, "pdd_solve_G: zero pivot in the dense LU of the system");
  return PDD_OK;
}

// Reports a final record through info and the return status.
pdd_status finish(const double* host, pdd_solve_info* info, const char* who) {
  const bool ok = host[S_DONE] != 0.0 && host[S_FAIL] == 0.0;
  const double bnorm = std::sqrt(host[S_BB]);
  const double rel = bnorm > 0.0 ? std::sqrt(host[S_RR]) / bnorm : 0.0;
  const int it = (int)host[S_ITER];
  if (info) {
    info->iterations = it;
    info->converged = ok ? 1 : 0;
    info->rel_residual = rel;
  }
  if (!ok)
    return fail(PDD_ENOCONV, std::string(who) + ": BiCGStab stopped at relative residual " +
                                 std::to_string(rel) + " after " + std::to_string(it) + " iterations");
  return PDD_OK;
}

}  // namespace

pdd_status solve_impl(pdd_system sys, const double* rhs, double* u, int32_t transpose,
                      const pdd_solve_opts* opts, hipStream_t st, pdd_solve_info* info) {
  const HostCover& H = sys->cover->H;
  const int64_t N = H.N();
  const SolveParams P = params(opts);
  const double* b = rhs ? rhs : sys->b.ptr<double>();
  if (P.method == PDD_SOLVE_DIRECT_SMALL) return direct_impl(sys, b, u, transpose != 0, st, info);
  if (P.method != PDD_SOLVE_BICGSTAB) return fail(PDD_EINVAL, "pdd_solve_G: unknown method");
  prepare_operator(sys, transpose != 0, st);
  const size_t wbytes = sizeof(double) * (size_t)work_doubles(N);
  // scratch from the cover's pool, returned when this call ends
  int dev = 0;
  PDD_HIP(hipGetDevice(&dev));
  std::unique_ptr<SolveScratch> scr;
  {
    std::lock_guard<std::mutex> lk(sys->cover->solve_mu);
    auto& pool = sys->cover->solve_free;
    for (size_t k = 0; k < pool.size(); ++k)
      if (pool[k]->device == dev) {
        scr = std::move(pool[k]);
        pool.erase(pool.begin() + k);
        break;
      }
  }
  if (!scr) {
    scr = std::make_unique<SolveScratch>();
    scr->device = dev;
  }
  struct Return {
    pdd_cover cv;
    hipStream_t q;
    std::unique_ptr<SolveScratch>& s;
    ~Return() {
      (void)hipStreamSynchronize(q);     // nothing in flight uses it (also on an error path)
      std::lock_guard<std::mutex> lk(cv->solve_mu);
      cv->solve_free.push_back(std::move(s));
    }
  } give_back{sys->cover, st, scr};
  if (scr->work.bytes() < wbytes) scr->work.alloc(wbytes);
  SolveCtx c{};
  bind(c, sys, transpose != 0, u, scr->work.ptr<double>());
  launch_init(c, b, P.guess, st);
  // Batches of kItersPerSync iterations; the convergence record of batch k is
  // copied to pinned host memory and read while batch k + 1 already runs (the
  // iteration kernels return at once after convergence, so a batch enqueued
  // past it does nothing).
  struct Pinned {
    double* p = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    ~Pinned() {
      for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    }
  } pin;
  if (!scr->pinned) PDD_HIP(hipHostMalloc(&scr->pinned, 2 * S_COUNT * sizeof(double), hipHostMallocDefault));
  pin.p = scr->pinned;
  for (int k = 0; k < 2 * S_COUNT; ++k) pin.p[k] = 0.0;
  for (auto& e : pin.ev) PDD_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  int enq = 0, slot = 0;
  auto batch_to = [&](int sl) {
    enq = enqueue_batch(c, st, enq, P.max_iter, P.rtol);
    PDD_HIP(hipMemcpyAsync(pin.p + sl * S_COUNT, c.status, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, st));
    PDD_HIP(hipEventRecord(pin.ev[sl], st));
  };
  batch_to(slot);
  for (;;) {
    const bool more = enq < P.max_iter;
    if (more) batch_to(slot ^ 1);
    PDD_HIP(hipEventSynchronize(pin.ev[slot]));
    const double* h = pin.p + slot * S_COUNT;
    if (h[S_DONE] != 0.0 || !more) break;
    slot ^= 1;
  }
  PDD_HIP(hipStreamSynchronize(st));
  // both slots now hold completed records; the more recent one (more
  // iterations counted; a batch that ran after convergence copies the same
  // record again) is the final state
  const double* a = pin.p;
  const double* b2 = pin.p + S_COUNT;
  return finish((b2[S_ITER] > a[S_ITER]) ? b2 : a, info, "pdd_solve_G");
}

// ------------------------------------------------- allocation-free variant

// Work area of pdd_solve_G_noalloc: 6 Mi doubles (48 MiB) of static device
// memory per GPU, held until the process ends.  In host code the name is only
// a stand-in: the device address comes from hipGetSymbolAddress.
constexpr int64_t kScratchDoubles = int64_t(6) << 20;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of `scratch` (looked up once per
// device, with that device current).
double* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    PDD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

pdd_status solve_noalloc_impl(pdd_system sys, const double* rhs, double* u, int32_t transpose,
                              const pdd_solve_opts* opts, hipStream_t st, pdd_solve_info* info) {
  const int64_t N = sys->cover->H.N();
  const SolveParams P = params(opts);
  if (P.method != PDD_SOLVE_BICGSTAB)
    return fail(PDD_EINVAL, "pdd_solve_G_noalloc: only PDD_SOLVE_BICGSTAB runs without allocating");
  if (work_doubles(N) > kScratchDoubles)
    return fail(PDD_EINVAL, "pdd_solve_G_noalloc: " + std::to_string(N) +
                                " unknowns need " + std::to_string(work_doubles(N)) +
                                " doubles of work area, more than its " + std::to_string(kScratchDoubles));
  {
    std::lock_guard<std::mutex> lk(sys->cover->solve_mu);
    if (!operator_ready(sys, transpose != 0))
      return fail(PDD_EINVAL, "pdd_solve_G_noalloc: the solve form of this system's operator has not "
                              "been built (one pdd_solve_G call in the same direction builds it)");
  }
  int dev = 0;
  PDD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PDD_EINVAL, "pdd_solve_G_noalloc: device index out of range");
  SolveCtx c{};
  bind(c, sys, transpose != 0, u, scratch_ptr(dev));
  const double* b = rhs ? rhs : sys->b.ptr<double>();
  launch_init(c, b, P.guess, st);
  // one stream synchronisation per batch of kItersPerSync iterations
  double host[S_COUNT];
  int enq = 0;
  for (;;) {
    enq = enqueue_batch(c, st, enq, P.max_iter, P.rtol);
    PDD_HIP(hipMemcpyAsync(host, c.status, sizeof host, hipMemcpyDeviceToHost, st));
    PDD_HIP(hipStreamSynchronize(st));
    if (host[S_DONE] != 0.0 || enq >= P.max_iter) break;
  }
  return finish(host, info, "pdd_solve_G_noalloc");
}

}  // namespace pdd

using namespace pdd;

extern "C" pdd_status pdd_solve_G_noalloc(pdd_system sys, const double* rhs, double* u, int32_t transpose,
                                          const pdd_solve_opts* opts, void* stream, pdd_solve_info* info) {
  if (!sys || !u) return fail(PDD_EINVAL, "pdd_solve_G_noalloc: null argument");
  try {
    return solve_noalloc_impl(sys, rhs, u, transpose, opts, (hipStream_t)stream, info);
  } catch (const HipError& e) {
    return fail(PDD_EDEVICE, e.what());
  } catch (const std::exception& e) {
    return fail(PDD_EDEVICE, std::string("pdd_solve_G_noalloc: ") + e.what());
  }
}

extern "C" pdd_status pdd_solve_G(pdd_system sys, const double* rhs, double* u, int32_t transpose,
                                  const pdd_solve_opts* opts, void* stream, pdd_solve_info* info) {
  if (!sys || !u) return fail(PDD_EINVAL, "pdd_solve_G: null argument");
  try {
    return solve_impl(sys, rhs, u, transpose, opts, (hipStream_t)stream, info);
  } catch (const HipError& e) {
    return fail(e.code == hipErrorOutOfMemory ? PDD_ENOMEM : PDD_EDEVICE, e.what());
  } catch (const std::bad_alloc&) {
    return fail(PDD_ENOMEM, "pdd_solve_G: out of host memory");
  } catch (const std::exception& e) {
    return fail(PDD_EDEVICE, std::string("pdd_solve_G: ") + e.what());
  }
}
