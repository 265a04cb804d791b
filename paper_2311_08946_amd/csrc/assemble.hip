// pdd_assemble_G: orchestration of the floating-row kernels (per size bucket
// and chunk), the Monte Carlo path and finalisation kernels and the boundary
// rows, followed by one status read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "mc.h"
#include "runtime.h"

namespace pdd {

namespace {

__global__ void reduce_u64_kernel(const uint64_t* __restrict__ a, int64_t n, uint64_t* out) {
  __shared__ uint64_t s[256];
  uint64_t v = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) v += a[i];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

// Rule AVERAGED (eqs. 38-39): row i of C is the rows of its pairs (knot i,
// circle m containing x_i) side by side, C_ii the number of pairs, r_i the sum
// of the pairs' r in pair order and its standard error their quadrature sum.
// One wavefront per knot; a pair row holds its diagonal slot first when the
// pair index is below the stencil's first knot, else last.
__global__ void __launch_bounds__(256) average_rows_kernel(
    int64_t N, const int64_t* __restrict__ pair_off, const int64_t* __restrict__ diag_pos,
    const int64_t* __restrict__ pair_seg, const int64_t* __restrict__ prowptr,
    const int32_t* __restrict__ passigned, const int64_t* __restrict__ knot_off,
    const double* __restrict__ pval, const double* __restrict__ pse, const double* __restrict__ pb,
    const double* __restrict__ pse_b, double* __restrict__ val, double* __restrict__ se,
    double* __restrict__ b, double* __restrict__ se_b) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= N) return;
  const int64_t p0 = pair_off[i], p1 = pair_off[i + 1];
  if (p0 == p1) return;   // boundary row, written by its own kernel
  double bs = 0.0, v2 = 0.0;
  for (int64_t p = p0; p < p1; ++p) {
    const int m = passigned[p];
    const int64_t lo = knot_off[m];
    const int M = (int)(knot_off[m + 1] - lo);
    const int64_t src = prowptr[p] + (p < lo ? 1 : 0);
    const int64_t dst = pair_seg[p];
    for (int c = lane; c < M; c += 64) {
      val[dst + c] = pval[src + c];
      se[dst + c] = pse[src + c];
    }
    bs += pb[p];
    v2 += pse_b[p] * pse_b[p];
  }
  if (lane == 0) {
    val[diag_pos[i]] = (double)(p1 - p0);
    se[diag_pos[i]] = 0.0;
    b[i] = bs;
    se_b[i] = sqrt(v2);
  }
}

__global__ void reduce_i32_kernel(const int32_t* __restrict__ a, int64_t n, uint64_t* out) {
  __shared__ uint64_t s[256];
  uint64_t v = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) v += (a[i] != 0);
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] += s[0];
}

struct PhaseTimer : PhaseHooks {
  hipStream_t st;
  struct Ev { int phase; hipEvent_t a, b; };
  std::vector<Ev> evs;
  explicit PhaseTimer(hipStream_t s) : st(s) {}
  ~PhaseTimer() {
    for (auto& e : evs) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
  }
  std::vector<hipStream_t> on;
  int begin(int phase, hipStream_t s = nullptr) override {
    Ev e{phase, nullptr, nullptr};
    PDD_HIP(hipEventCreate(&e.a));
    PDD_HIP(hipEventCreate(&e.b));
    hipStream_t q = s ? s : st;
    PDD_HIP(hipEventRecord(e.a, q));
    evs.push_back(e);
    on.push_back(q);
    return (int)evs.size() - 1;
  }
  void end(int idx) override { PDD_HIP(hipEventRecord(evs[idx].b, on[idx])); }
  float total(int phase) {
    float t = 0.0f;
    for (auto& e : evs)
      if (e.phase == phase) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) t += ms;
      }
    return t;
  }
};

__global__ void eval_field_kernel(const DevProblem* __restrict__ P, int which,
                                  const double* __restrict__ xy, int64_t n, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = xy[2 * i], y = xy[2 * i + 1];
  double v;
  if (which < 7) {
    double co[7];
    coefficients_at(*P, x, y, co);
    v = co[which];
  } else if (which == 7) {
    v = boundary_value(*P, x, y);
  } else {
    v = field_plain(P->fld[F_U], x, y);
  }
  out[i] = v;
}

}  // namespace

void alloc_factors(BucketFactors& f, const BucketData& bk, int32_t count) {
  f.stride = (int64_t)bk.n * bk.ld;
  f.A.alloc((size_t)count * f.stride * sizeof(double));
  f.piv.alloc((size_t)count * bk.n * sizeof(int32_t));
  f.rowscale.alloc((size_t)count * bk.n * sizeof(double));
  f.status.alloc((size_t)count * sizeof(int32_t));
}

int factor_chunk(const DeviceCover& D, const BucketData& bk, const NodeSamples& S, int plan,
                 BucketFactors& f, int32_t first, int32_t cnt, LuScratch& ws, hipStream_t st,
                 PhaseHooks* hooks, double* val, double* b) {
  const size_t wbytes = lu_workspace_bytes(plan == PDD_PLAN_PER_CIRCLE ? 1 : cnt, bk.n);
  if (ws.bytes < wbytes) {
    PDD_HIP(hipStreamSynchronize(st));
    ws.buf.alloc(wbytes);
    ws.bytes = wbytes;
  }
  f.first = first;
  f.count = cnt;
  const int64_t stride = f.stride;
  int launches = 0;
  const int32_t step = (plan == PDD_PLAN_PER_CIRCLE) ? 1 : cnt;
  for (int32_t s0 = 0; s0 < cnt; s0 += step) {
    const int32_t c1 = std::min(step, cnt - s0);
    ChunkDesc C = D.chunk(bk, first + s0, c1);
    double* A = f.A.ptr<double>() + (int64_t)s0 * stride;
    int e = hooks ? hooks->begin(PH_BUILD) : -1;
    launch_colloc_build(bk.T, C, S, A, stride, f.rowscale.ptr<double>() + (int64_t)s0 * bk.n, st);
    if (hooks) hooks->end(e);
    e = hooks ? hooks->begin(PH_LU) : -1;
    launches += 1 + launch_lu_solve(bk.T, c1, A, stride, f.piv.ptr<int32_t>() + (int64_t)s0 * bk.n,
                                    f.status.ptr<int32_t>() + s0, ws.buf.ptr<void>(), st);
    if (hooks) hooks->end(e);
    if (val) {
      e = hooks ? hooks->begin(PH_EVAL) : -1;
      launch_eval_scatter(bk.T, C, A, stride, val, b, st);
      if (hooks) hooks->end(e);
      ++launches;
    }
  }
  PDD_HIP(hipGetLastError());
  return launches;
}

// ---------------------------------------------------------------------------
// Schedule of the floating circles: groups of bucket slices, one persistent LU
// launch sequence per group.

struct Slice {
  int32_t bucket, first, cnt;
};

struct Schedule {
  bool mixed = true;
  int grid_cap = 0;          // multiple of the compute units; 0 = one workgroup per tile
  bool graph = false;
  bool lookahead = true;     // U-row tiles of step s beside the panel of step s + 1
};

// Groups of circles whose factors are resident together.
std::vector<std::vector<Slice>> make_groups(const DeviceCover& D, int plan, bool keep_all, int64_t budget,
                                            bool mixed) {
  std::vector<std::vector<Slice>> groups;
  const int nb = (int)D.buckets.size();
  if (plan == PDD_PLAN_PER_CIRCLE) {
    for (int b = 0; b < nb; ++b)
      for (int32_t i = 0; i < D.buckets[b]->count; ++i) groups.push_back({Slice{b, i, 1}});
    return groups;
  }
  if (!mixed) {
    for (int b = 0; b < nb; ++b) {
      const BucketData& bk = *D.buckets[b];
      const int32_t chunk = keep_all ? bk.count
                                     : (int32_t)std::min<int64_t>(bk.count,
                                                                  std::max<int64_t>(1, budget / factor_bytes_per_circle(bk)));
      for (int32_t first = 0; first < bk.count; first += chunk)
        groups.push_back({Slice{b, first, std::min(chunk, bk.count - first)}});
    }
    return groups;
  }
  int64_t total = 0, most = 1;
  for (int b = 0; b < nb; ++b) {
    total += (int64_t)D.buckets[b]->count * factor_bytes_per_circle(*D.buckets[b]);
    most = std::max<int64_t>(most, D.buckets[b]->count);
  }
  // a group holds the same share of every bucket; the number of groups G
  // grows geometrically until the largest group fits the budget, and stops at
  // one circle per bucket and group
  int64_t G = keep_all ? 1 : std::min(most, std::max<int64_t>(1, (total + budget - 1) / budget));
  while (!keep_all && G < most) {
    int64_t worst = 0;
    for (int64_t g = 0; g < G; ++g) {
      int64_t bytes = 0;
      for (int b = 0; b < nb; ++b) {
        const int64_t c = D.buckets[b]->count;
        bytes += (c * (g + 1) / G - c * g / G) * factor_bytes_per_circle(*D.buckets[b]);
      }
      worst = std::max(worst, bytes);
    }
    if (worst <= budget) break;
    G = std::min(most, std::max(G + 1, G + G / 4));
  }
  for (int64_t g = 0; g < G; ++g) {
    std::vector<Slice> grp;
    for (int b = 0; b < nb; ++b) {
      const int64_t c = D.buckets[b]->count;
      const int32_t lo = (int32_t)(c * g / G), hi = (int32_t)(c * (g + 1) / G);
      if (hi > lo) grp.push_back(Slice{b, lo, hi - lo});
    }
    if (!grp.empty()) groups.push_back(std::move(grp));
  }
  return groups;
}

// Runs groups: build launches per slice, the group's LU plan (replayed from a
// captured graph when the previous group had the same shape and buffers),
// evaluation launches per slice.
struct GroupRun {
  const DeviceCover& D;
  hipStream_t st;
  Schedule sched;
  int cus = 256;
  LuScratch work;
  std::vector<std::unique_ptr<BucketFactors>> reuse;   // per bucket, transient groups
  std::vector<std::unique_ptr<LuPlan>> plans;          // alive as long as the run
  struct Planned {
    std::vector<int32_t> counts;
    std::vector<BucketFactors*> fs;
    LuPlan* plan;
  };
  std::vector<Planned> planned;
  LuPlan* last_plan = nullptr;
  std::vector<int32_t> last_counts;
  std::vector<BucketFactors*> last_fs;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int replays = 0;

  GroupRun(const DeviceCover& d, hipStream_t s, const Schedule& sc) : D(d), st(s), sched(sc) {
    int dev = 0;
    PDD_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    PDD_HIP(hipGetDeviceProperties(&prop, dev));
    cus = prop.multiProcessorCount;
    reuse.resize(D.buckets.size());
  }
  ~GroupRun() { drop_graph(); if (cap_stream) (void)hipStreamDestroy(cap_stream); }

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }

  BucketFactors* reusable(int b, const std::vector<std::vector<Slice>>& groups) {
    if (!reuse[b]) {
      int32_t most = 1;
      for (const auto& g : groups)
        for (const auto& sl : g)
          if (sl.bucket == b) most = std::max(most, sl.cnt);
      reuse[b] = std::make_unique<BucketFactors>();
      reuse[b]->bucket = b;
      alloc_factors(*reuse[b], *D.buckets[b], most);
    }
    return reuse[b].get();
  }

  int grid_cap() const { return sched.grid_cap > 0 ? sched.grid_cap * cus : (1 << 30); }

  int group(const std::vector<Slice>& grp, const std::vector<BucketFactors*>& fs, const NodeSamples& S,
            PhaseHooks* hooks, double* val, double* b, uint64_t* fail_count) {
    int launches = 0;
    size_t wbytes = 0;
    for (const auto& sl : grp) wbytes += (size_t)sl.cnt * lu_work_bytes_per_matrix(D.buckets[sl.bucket]->n);
    if (work.bytes < wbytes) {
      PDD_HIP(hipStreamSynchronize(st));
      drop_graph();
      last_plan = nullptr;
      planned.clear();                     // their items point into the old work buffer
      work.buf.alloc(wbytes);
      work.bytes = wbytes;
    }
    int e = hooks ? hooks->begin(PH_BUILD) : -1;
    for (size_t k = 0; k < grp.size(); ++k) {
      const BucketData& bk = *D.buckets[grp[k].bucket];
      ChunkDesc C = D.chunk(bk, grp[k].first, grp[k].cnt);
      launch_colloc_build(bk.T, C, S, fs[k]->A.ptr<double>(), fs[k]->stride, fs[k]->rowscale.ptr<double>(), st);
      ++launches;
    }
    if (hooks) hooks->end(e);
    // the group's matrices, in slice order
    std::vector<int32_t> counts;
    for (const auto& sl : grp) counts.push_back(sl.bucket), counts.push_back(sl.cnt);
    const bool same = last_plan && counts == last_counts && fs == last_fs;
    // a group this run has planned before (the autotuner repeats its groups)
    LuPlan* seen = nullptr;
    if (!same)
      for (const auto& pk : planned)
        if (pk.counts == counts && pk.fs == fs) seen = pk.plan;
    e = hooks ? hooks->begin(PH_LU) : -1;
    if (seen) {
      launches += seen->launch(st, grid_cap(), sched.lookahead);
    } else if (!same) {
      std::vector<LuItem> its;
      char* w = static_cast<char*>(work.buf.ptr<void>());
      for (size_t k = 0; k < grp.size(); ++k) {
        const BucketData& bk = *D.buckets[grp[k].bucket];
        const size_t per = lu_work_bytes_per_matrix(bk.n);
        for (int32_t i = 0; i < grp[k].cnt; ++i) {
          LuItem it;
          it.A = fs[k]->A.ptr<double>() + (int64_t)i * fs[k]->stride;
          it.piv = fs[k]->piv.ptr<int32_t>() + (int64_t)i * bk.n;
          it.status = fs[k]->status.ptr<int32_t>() + i;
          it.work = reinterpret_cast<LuWork*>(w);
          it.uinv = reinterpret_cast<double*>(w + lu_work_header_bytes());
          it.n = bk.n;
          it.ld = bk.ld;
          it.nrhs = bk.nrhs;
          it.cls = lu_panel_class(bk.n);
          its.push_back(it);
          w += per;
        }
      }
      auto plan = std::make_unique<LuPlan>();
      plan->build(its);
      last_plan = plan.get();
      planned.push_back(Planned{counts, fs, plan.get()});
      plans.push_back(std::move(plan));
      last_counts = counts;
      last_fs = fs;
      drop_graph();
      if (sched.graph) {
        if (!cap_stream) PDD_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
        PDD_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
        last_plan->launch(cap_stream, grid_cap(), sched.lookahead);
        PDD_HIP(hipStreamEndCapture(cap_stream, &graph));
        PDD_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        PDD_HIP(hipGraphLaunch(exec, st));
        launches += 1;
      } else {
        launches += last_plan->launch(st, grid_cap(), sched.lookahead);
      }
    } else if (exec) {
      PDD_HIP(hipGraphLaunch(exec, st));
      ++replays;
      launches += 1;
    } else {
      launches += last_plan->launch(st, grid_cap(), sched.lookahead);
    }
    if (hooks) hooks->end(e);
    if (val) {
      e = hooks ? hooks->begin(PH_EVAL) : -1;
      for (size_t k = 0; k < grp.size(); ++k) {
        const BucketData& bk = *D.buckets[grp[k].bucket];
        ChunkDesc C = D.chunk(bk, grp[k].first, grp[k].cnt);
        launch_eval_scatter(bk.T, C, fs[k]->A.ptr<double>(), fs[k]->stride, val, b, st);
        ++launches;
      }
      if (hooks) hooks->end(e);
    }
    for (size_t k = 0; k < grp.size(); ++k)
      hipLaunchKernelGGL(reduce_i32_kernel, dim3(1), dim3(256), 0, st, fs[k]->status.ptr<int32_t>(),
                         (int64_t)grp[k].cnt, fail_count);
    PDD_HIP(hipGetLastError());
    return launches;
  }

  void finish() { PDD_HIP(hipStreamSynchronize(st)); }
};

// Times the candidate schedules (mixed or per-bucket groups, grid caps) on a
// sample of each bucket (build and LU) and returns the fastest.  The sample
// is large enough to fill the GPU several times over (up to 2048 circles per
// bucket, at most 8 GiB of factors in all), every candidate's plan is built
// and run once untimed, then its launches are timed three times and the
// median kept.  With one bucket the mixed and per-bucket groupings are the
// same schedule and only the grid caps are compared.
void autotune(const DeviceCover& D, const NodeSamples& S, int64_t budget, hipStream_t st, bool& mixed,
              int& cap, bool& lookahead) {
  constexpr int kSampleMax = 2048;
  constexpr int64_t kSampleBytes = (int64_t)8 << 30;
  std::vector<std::vector<Slice>> sample_mixed(1), sample_sep;
  int64_t per_bucket_bytes = kSampleBytes / std::max<int64_t>(1, (int64_t)D.buckets.size());
  for (int b = 0; b < (int)D.buckets.size(); ++b) {
    const int64_t fit = std::max<int64_t>(1, per_bucket_bytes / factor_bytes_per_circle(*D.buckets[b]));
    const int32_t c = (int32_t)std::min<int64_t>({(int64_t)kSampleMax, fit, (int64_t)D.buckets[b]->count});
    if (c == 0) continue;
    sample_mixed[0].push_back(Slice{b, 0, c});
    sample_sep.push_back({Slice{b, 0, c}});
  }
  std::vector<std::unique_ptr<BucketFactors>> fac(D.buckets.size());
  for (const auto& sl : sample_mixed[0]) {
    fac[sl.bucket] = std::make_unique<BucketFactors>();
    fac[sl.bucket]->bucket = sl.bucket;
    alloc_factors(*fac[sl.bucket], *D.buckets[sl.bucket], sl.cnt);
  }
  DevBuf fails;
  fails.alloc(sizeof(uint64_t));
  hipEvent_t e0, e1;
  PDD_HIP(hipEventCreate(&e0));
  PDD_HIP(hipEventCreate(&e1));
  struct Guard {
    hipEvent_t a, b;
    ~Guard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  } guard{e0, e1};
  float best = 1e30f;
  const int caps[3] = {0, 1, 2};
  const bool one_bucket = sample_sep.size() <= 1;
  for (int mx = 1; mx >= (one_bucket ? 1 : 0); --mx)
    for (int la = 1; la >= 0; --la)
    for (int ci = 0; ci < 3; ++ci) {
      Schedule sc;
      sc.mixed = mx != 0;
      sc.grid_cap = caps[ci];
      sc.lookahead = la != 0;
      const auto& groups = sc.mixed ? sample_mixed : sample_sep;
      GroupRun run(D, st, sc);
      auto once = [&]() {
        for (const auto& grp : groups) {
          std::vector<BucketFactors*> fs;
          for (const auto& sl : grp) fs.push_back(fac[sl.bucket].get());
          run.group(grp, fs, S, nullptr, nullptr, nullptr, fails.ptr<uint64_t>());
        }
      };
      once();                                   // builds the plans, first-touch costs
      once();                                   // (groups planned before a work-buffer growth)
      run.finish();
      float ms[3];
      for (int rep = 0; rep < 3; ++rep) {
        PDD_HIP(hipEventRecord(e0, st));
        once();
        PDD_HIP(hipEventRecord(e1, st));
        run.finish();
        PDD_HIP(hipEventElapsedTime(&ms[rep], e0, e1));
      }
      std::sort(ms, ms + 3);
      if (ms[1] < best) {
        best = ms[1];
        mixed = sc.mixed;
        cap = sc.grid_cap;
        lookahead = sc.lookahead;
      }
    }
  (void)budget;
}

pdd_status assemble_impl(pdd_cover cover, const pdd_problem* problem, const pdd_samples* samples,
                         const pdd_mc_opts* mc, const pdd_assemble_opts* opts, hipStream_t st,
                         pdd_system* out) {
  const HostCover& H0 = cover->H;
  const bool avg = H0.pairs != nullptr;
  const HostCover& H = avg ? *H0.pairs : H0;   // the rows the kernels assemble
  if (!H.mc_knots.empty()) {
    if (!mc) return fail(PDD_EINVAL, "pdd_assemble_G: Monte Carlo options are required");
    if (mc->paths < 2 || !(mc->h > 0.0) || mc->n_batches < 2 || mc->n_batches > 63 ||
        mc->step_cap <= 0 || mc->paths < mc->n_batches || mc->paths > ((int64_t)1 << 32) ||
        mc->scheme < PDD_MC_EULER || mc->scheme > PDD_MC_SHIFTED)
      return fail(PDD_EINVAL, "pdd_assemble_G: bad Monte Carlo options");
    const int64_t tri = (int64_t)H.max_arc * (H.max_arc + 1) / 2;
    if ((tri + (int64_t)(mc->n_batches + 1) * H.max_arc) * (int64_t)sizeof(double) > 160 * 1024)
      return fail(PDD_EINVAL, "pdd_assemble_G: arc length and batch count exceed the 160 KiB LDS budget "
                              "of the Monte Carlo finalisation");
  }
  int dev = 0;
  PDD_HIP(hipGetDevice(&dev));
  DeviceCover& D0 = cover->D;
  if (!D0.ready || D0.device != dev) {
    D0.upload(H0);
    D0.device = dev;
  }
  DeviceCover& D = avg ? cover->DP : D0;
  if (avg && (!D.ready || D.device != dev)) {
    D.upload(H);
    D.device = dev;
  }
  auto sys = std::make_unique<pdd_system_s>();
  sys->cover = cover;
  const int64_t N0 = H0.N(), nnz0 = H0.rowptr.back();
  sys->val.alloc(nnz0 * sizeof(double));
  sys->se.alloc(nnz0 * sizeof(double));
  sys->b.alloc(N0 * sizeof(double));
  sys->se_b.alloc(N0 * sizeof(double));
  PDD_HIP(hipMemsetAsync(sys->se.ptr<void>(), 0, nnz0 * sizeof(double), st));
  PDD_HIP(hipMemsetAsync(sys->se_b.ptr<void>(), 0, N0 * sizeof(double), st));
  // the rows the kernels write: those of C, or under rule AVERAGED the pair
  // rows, combined into C at the end
  DevBuf pair_val, pair_se, pair_b, pair_se_b;
  double *val = sys->val.ptr<double>(), *se = sys->se.ptr<double>();
  double *bv = sys->b.ptr<double>(), *se_b = sys->se_b.ptr<double>();
  if (avg) {
    const int64_t np = H.N(), nnzp = H.rowptr.back();
    pair_val.alloc(std::max<int64_t>(1, nnzp) * sizeof(double));
    pair_se.alloc(std::max<int64_t>(1, nnzp) * sizeof(double));
    pair_b.alloc(std::max<int64_t>(1, np) * sizeof(double));
    pair_se_b.alloc(std::max<int64_t>(1, np) * sizeof(double));
    PDD_HIP(hipMemsetAsync(pair_se.ptr<void>(), 0, std::max<int64_t>(1, nnzp) * sizeof(double), st));
    PDD_HIP(hipMemsetAsync(pair_se_b.ptr<void>(), 0, std::max<int64_t>(1, np) * sizeof(double), st));
    val = pair_val.ptr<double>();
    se = pair_se.ptr<double>();
    bv = pair_b.ptr<double>();
    se_b = pair_se_b.ptr<double>();
  }

  DevProblem dp;
  pdd_status ps = make_dev_problem(*problem, dp);
  if (ps != PDD_OK) return ps;
  sys->problem.alloc(sizeof(DevProblem));
  PDD_HIP(hipMemcpy(sys->problem.ptr<void>(), &dp, sizeof(DevProblem), hipMemcpyHostToDevice));
  const DevProblem* P = sys->problem.ptr<DevProblem>();

  const int plan = opts ? opts->plan : PDD_PLAN_BATCHED;
  const bool keep = opts ? opts->keep_factors != 0 : false;
  const int64_t budget = (opts && opts->hbm_budget_bytes > 0) ? opts->hbm_budget_bytes
                                                              : (int64_t)64 << 30;
  int64_t factor_total = 0;
  for (auto& bp : D.buckets) factor_total += (int64_t)bp->count * factor_bytes_per_circle(*bp);
  const bool keep_all = keep && factor_total <= budget;
  sys->recompute = keep && !keep_all;
  sys->budget = budget;
  sys->plan = plan;
  PhaseTimer timer(st);
  const int t_all = timer.begin(PH_TOTAL);

  // ---- node samples
  const int64_t sum_n = H.sum_n;
  NodeSamples S{};
  const double* given[7] = {nullptr};
  if (samples) {
    const double* g[7] = {samples->axx, samples->axy, samples->ayy, samples->bx,
                          samples->by,  samples->c,   samples->f};
    for (int t = 0; t < 7; ++t) given[t] = g[t];
  }
  bool need = false;
  for (int t = 0; t < 7; ++t) need = need || !given[t];
  // a system whose factors are recomputed in the backward pass keeps its own
  // copy of every sample
  if ((need || sys->recompute) && sum_n > 0) sys->samples.alloc(7 * sum_n * sizeof(double));
  for (int t = 0; t < 7; ++t) {
    double* own = (need || sys->recompute) && sum_n > 0 ? sys->samples.ptr<double>() + (int64_t)t * sum_n : nullptr;
    if (given[t] && own)
      PDD_HIP(hipMemcpyAsync(own, given[t], sum_n * sizeof(double), hipMemcpyDeviceToDevice, st));
    S.s[t] = own ? own : given[t];
  }
  if (need && sum_n > 0) {
    const int ev = timer.begin(PH_SAMPLE);
    double* outs[7];
    for (int t = 0; t < 7; ++t) outs[t] = given[t] ? nullptr : const_cast<double*>(S.s[t]);
    for (auto& bp : D.buckets) {
      ChunkDesc C = D.chunk(*bp, 0, bp->count);
      launch_sample_nodes(P, bp->T, C, outs, st);
    }
    PDD_HIP(hipGetLastError());
    timer.end(ev);
  }

  // ---- schedule of the floating rows (tuned before the Monte Carlo work starts)
  Schedule sched;
  sched.mixed = opts ? opts->mixed_buckets != 0 : true;
  sched.grid_cap = opts ? std::max(0, opts->grid_cap) : 0;
  sched.graph = opts ? opts->use_graph != 0 : false;
  sched.lookahead = opts ? opts->no_lookahead == 0 : true;
  float ms_tune = 0.0f;
  if (plan == PDD_PLAN_AUTOTUNED) {
    if (!D.tuned) {
      const auto t0 = std::chrono::steady_clock::now();
      autotune(D, S, budget, st, D.tuned_mixed, D.tuned_cap, D.tuned_lookahead);
      D.tuned = true;
      ms_tune = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    sched.mixed = D.tuned_mixed;
    sched.grid_cap = D.tuned_cap;
    sched.lookahead = D.tuned_lookahead;
  }
  // The Monte Carlo and boundary rows run on a second stream, concurrently
  // with the floating rows; both write disjoint rows of the CSR arrays.  When
  // the last autotuned assembly on this cover found the Monte Carlo work about
  // as long as the floating rows, the floating rows gained nothing beside it
  // (their panels need whole CUs, which its workgroups keep refilling): it
  // then starts after them.
  DevBuf lu_fail;
  lu_fail.alloc(sizeof(uint64_t) * 5);
  PDD_HIP(hipMemsetAsync(lu_fail.ptr<void>(), 0, sizeof(uint64_t) * 5, st));
  if (!D.side) PDD_HIP(hipStreamCreateWithFlags(&D.side, hipStreamNonBlocking));
  hipStream_t side = D.side;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  PDD_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
  PDD_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  } ev_guard{ev_fork, ev_join};
  const int mc_order = opts ? opts->mc_order : 0;
  if (mc_order < 0 || mc_order > 2) return fail(PDD_EINVAL, "mc_order must be 0, 1 or 2");
  const bool mc_after = mc_order == 2 || (mc_order == 0 && plan == PDD_PLAN_AUTOTUNED && D.last_ms_mc > 0.0f &&
                                          D.last_ms_mc >= 0.8f * D.last_ms_float);

  // ---- perimeter rows by Monte Carlo (side stream)
  const int64_t n_mc = (int64_t)H.mc_knots.size();
  const int64_t n_perim = (int64_t)H.perim_ids.size();
  DevBuf out_phi, out_g, out_steps, out_capped, out_gamma, gram, gram_status, hcirc;
  int32_t n_launch_mc = 0;
  auto mc_rows = [&]() {
    PDD_HIP(hipEventRecord(ev_fork, st));
    PDD_HIP(hipStreamWaitEvent(side, ev_fork, 0));
    if (n_mc > 0) {
      const int e = timer.begin(PH_MC, side);
      McArgs a{};
      a.mc_knots = D.mc_knots.ptr<int32_t>();
      a.assigned = D.assigned.ptr<int32_t>();
      a.perim_ids = D.perim_ids.ptr<int32_t>();
      a.perim_pos = D.perim_pos.ptr<int32_t>();
      a.cx = D.cx.ptr<double>(); a.cy = D.cy.ptr<double>(); a.rad = D.rad.ptr<double>();
      a.arc0 = D.arc0.ptr<double>(); a.arc1 = D.arc1.ptr<double>(); a.rbf_c2 = D.rbf_c2.ptr<double>();
      a.knot_off = D.knot_off.ptr<int64_t>();
      a.kx = D.kx.ptr<double>(); a.ky = D.ky.ptr<double>(); a.ktheta = D.ktheta.ptr<double>();
      a.rowptr = D.rowptr.ptr<int64_t>();
      if (mc->h_per_circle) {
        std::vector<double> hv(mc->h_per_circle, mc->h_per_circle + H.nc);
        hcirc.upload(hv);
        a.h_circle = hcirc.ptr<double>();
      }
      a.h = mc->h;
      a.seed = mc->seed;
      a.paths = mc->paths;
      a.n_batches = mc->n_batches;
      a.step_cap = mc->step_cap;
      a.scheme = mc->scheme;
      a.n_units = n_mc * mc->n_batches;
      a.out_stride = std::max<int64_t>(1, H.max_arc);
      a.gram_stride = (int64_t)H.max_arc * (H.max_arc + 1) / 2;
      out_phi.alloc(std::max<int64_t>(1, a.n_units * a.out_stride) * sizeof(double));
      out_g.alloc(std::max<int64_t>(1, a.n_units) * sizeof(double));
      out_steps.alloc(std::max<int64_t>(1, a.n_units) * sizeof(uint64_t));
      out_capped.alloc(std::max<int64_t>(1, a.n_units) * sizeof(uint64_t));
      out_gamma.alloc(std::max<int64_t>(1, a.n_units) * sizeof(uint64_t));
      gram.alloc(std::max<int64_t>(1, n_perim * a.gram_stride) * sizeof(double));
      gram_status.alloc(std::max<int64_t>(1, n_perim) * sizeof(int32_t));
      a.out_phi = out_phi.ptr<double>();
      a.out_g = out_g.ptr<double>();
      a.out_steps = out_steps.ptr<uint64_t>();
      a.out_capped = out_capped.ptr<uint64_t>();
      a.out_gamma = out_gamma.ptr<uint64_t>();
      launch_mc_paths(P, dp, a, side);
      launch_gram_cholesky(a, (int32_t)n_perim, gram.ptr<double>(), gram_status.ptr<int32_t>(), side);
      launch_mc_finalize(a, (int32_t)n_mc, H.max_arc, gram.ptr<double>(), val, se, bv, se_b, side);
      PDD_HIP(hipGetLastError());
      hipLaunchKernelGGL(reduce_u64_kernel, dim3(1), dim3(256), 0, side, out_steps.ptr<uint64_t>(),
                         a.n_units, lu_fail.ptr<uint64_t>() + 1);
      hipLaunchKernelGGL(reduce_u64_kernel, dim3(1), dim3(256), 0, side, out_capped.ptr<uint64_t>(),
                         a.n_units, lu_fail.ptr<uint64_t>() + 2);
      if (n_perim > 0)
        hipLaunchKernelGGL(reduce_i32_kernel, dim3(1), dim3(256), 0, side, gram_status.ptr<int32_t>(),
                           n_perim, lu_fail.ptr<uint64_t>() + 3);
      hipLaunchKernelGGL(reduce_u64_kernel, dim3(1), dim3(256), 0, side, out_gamma.ptr<uint64_t>(),
                         a.n_units, lu_fail.ptr<uint64_t>() + 4);
      n_launch_mc = 3;
      timer.end(e);
    }
    launch_boundary_rows(P, D0.bnd_knots.ptr<int32_t>(), (int32_t)H0.bnd_knots.size(), D0.kx.ptr<double>(),
                         D0.ky.ptr<double>(), D0.rowptr.ptr<int64_t>(), sys->val.ptr<double>(),
                         sys->se.ptr<double>(), sys->b.ptr<double>(), sys->se_b.ptr<double>(), side);
    PDD_HIP(hipGetLastError());
    PDD_HIP(hipEventRecord(ev_join, side));
  };
  if (!mc_after) mc_rows();

  // ---- floating rows in groups (see the schedule in pdd.h)
  const auto groups = make_groups(D, plan, keep_all, budget, sched.mixed);
  // a captured graph pays only when later groups replay it: groups of the same
  // shape on the same transient buffers (stored factors give every group its own)
  if (keep_all || groups.size() < 2) sched.graph = false;
  GroupRun run(D, st, sched);
  int32_t n_launch_spectral = 0;
  int64_t kept = 0;
  for (const auto& grp : groups) {
    std::vector<BucketFactors*> fs(grp.size());
    for (size_t k = 0; k < grp.size(); ++k) {
      const Slice& sl = grp[k];
      if (keep_all) {
        auto f = std::make_unique<BucketFactors>();
        f->bucket = sl.bucket;
        alloc_factors(*f, *D.buckets[sl.bucket], sl.cnt);
        f->first = sl.first;
        f->count = sl.cnt;
        fs[k] = f.get();
        kept += (int64_t)sl.cnt * factor_bytes_per_circle(*D.buckets[sl.bucket]);
        sys->factors.push_back(std::move(f));
      } else {
        fs[k] = run.reusable(sl.bucket, groups);
        fs[k]->first = sl.first;
        fs[k]->count = sl.cnt;
      }
    }
    n_launch_spectral += run.group(grp, fs, S, &timer, val, bv, lu_fail.ptr<uint64_t>());
  }
  run.finish();
  if (mc_after) mc_rows();

  PDD_HIP(hipStreamWaitEvent(st, ev_join, 0));
  if (avg && N0 > 0) {
    hipLaunchKernelGGL(average_rows_kernel, dim3((unsigned)((N0 + 3) / 4)), dim3(256), 0, st, N0,
                       D0.pair_off.ptr<int64_t>(), D0.diag_pos.ptr<int64_t>(),
                       D.pair_seg.ptr<int64_t>(), D.rowptr.ptr<int64_t>(), D.assigned.ptr<int32_t>(),
                       D.knot_off.ptr<int64_t>(), val, se, bv, se_b, sys->val.ptr<double>(),
                       sys->se.ptr<double>(), sys->b.ptr<double>(), sys->se_b.ptr<double>());
    PDD_HIP(hipGetLastError());
  }
  timer.end(t_all);

  uint64_t flags[5] = {0, 0, 0, 0, 0};
  PDD_HIP(hipMemcpyAsync(flags, lu_fail.ptr<void>(), sizeof(flags), hipMemcpyDeviceToHost, st));
  PDD_HIP(hipStreamSynchronize(st));
  pdd_system_stats& s = sys->stats;
  s.path_steps = (int64_t)flags[1];
  s.capped_paths = (int64_t)flags[2];
  s.gamma_exits = (int64_t)flags[4];
  s.paths = mc ? n_mc * mc->paths : 0;
  s.breakdowns = (int32_t)(flags[0] + flags[3]);
  s.n_launch_spectral = n_launch_spectral;
  s.factor_bytes = kept;
  s.recompute = sys->recompute ? 1 : 0;
  s.n_groups = (int32_t)groups.size();
  s.mixed_buckets = sched.mixed ? 1 : 0;
  s.grid_cap = sched.grid_cap;
  s.lu_lookahead = sched.lookahead ? 1 : 0;
  s.mc_after_floating = mc_after ? 1 : 0;
  s.graph_replays = run.replays;
  s.ms_autotune = ms_tune;
  s.n_launch_mc = n_launch_mc;
  s.ms_sample = timer.total(PH_SAMPLE);
  s.ms_build = timer.total(PH_BUILD);
  s.ms_lu = timer.total(PH_LU);
  s.ms_solve = timer.total(PH_SOLVE);
  s.ms_eval = timer.total(PH_EVAL);
  s.ms_mc = timer.total(PH_MC);
  s.ms_total = timer.total(PH_TOTAL);
  if (plan == PDD_PLAN_AUTOTUNED) {
    D.last_ms_mc = s.ms_mc;
    D.last_ms_float = s.ms_sample + s.ms_build + s.ms_lu + s.ms_eval;
  }
  if (s.breakdowns) {
    *out = sys.release();
    return fail(PDD_EBREAKDOWN, "pdd_assemble_G: zero pivot in a collocation LU or non-SPD Gram matrix");
  }
  if (s.capped_paths) {
    *out = sys.release();
    return fail(PDD_EPATHCAP, "pdd_assemble_G: " + std::to_string(s.capped_paths) +
                                  " paths exceeded the step cap");
  }
  *out = sys.release();
  return PDD_OK;
}

}  // namespace pdd

using namespace pdd;

extern "C" {

pdd_status pdd_assemble_G(pdd_cover cover, const pdd_problem* problem, const pdd_samples* samples,
                          const pdd_mc_opts* mc, const pdd_assemble_opts* opts, void* stream,
                          pdd_system* out) {
  if (!cover || !problem || !out) return fail(PDD_EINVAL, "pdd_assemble_G: null argument");
  *out = nullptr;
  try {
    return assemble_impl(cover, problem, samples, mc, opts, (hipStream_t)stream, out);
  } catch (const HipError& e) {
    return fail(e.code == hipErrorOutOfMemory ? PDD_ENOMEM : PDD_EDEVICE, e.what());
  } catch (const std::bad_alloc&) {
    return fail(PDD_ENOMEM, "pdd_assemble_G: out of host memory");
  } catch (const std::exception& e) {
    return fail(PDD_EDEVICE, e.what());
  }
}

pdd_status pdd_eval_field(const pdd_problem* problem, int32_t which, const double* xy, int64_t n,
                          double* out, void* stream) {
  if (!problem || (n > 0 && (!xy || !out)) || which < 0 || which > PDD_WHICH_U || n < 0)
    return fail(PDD_EINVAL, "pdd_eval_field: bad argument");
  try {
    DevProblem dp;
    pdd_status ps = make_dev_problem(*problem, dp);
    if (ps != PDD_OK) return ps;
    if (which == PDD_WHICH_U && dp.fld[F_U].kind == PDD_FIELD_DERIVED_F)
      return fail(PDD_EINVAL, "pdd_eval_field: u cannot be a derived field");
    if (n == 0) return PDD_OK;
    hipStream_t st = (hipStream_t)stream;
    DevBuf pb;
    pb.alloc(sizeof(DevProblem));
    PDD_HIP(hipMemcpyAsync(pb.ptr<void>(), &dp, sizeof(DevProblem), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(eval_field_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       pb.ptr<DevProblem>(), (int)which, xy, n, out);
    PDD_HIP(hipGetLastError());
    PDD_HIP(hipStreamSynchronize(st));
    return PDD_OK;
  } catch (const HipError& e) {
    return fail(PDD_EDEVICE, e.what());
  } catch (const std::bad_alloc&) {
    return fail(PDD_ENOMEM, "pdd_eval_field: out of host memory");
  } catch (const std::exception& e) {
    return fail(PDD_EDEVICE, std::string("pdd_eval_field: ") + e.what());
  }
}

pdd_status pdd_system_copy(pdd_system sys, double* val, double* b, double* se, double* se_b,
                           void* stream) {
  if (!sys) return fail(PDD_EINVAL, "pdd_system_copy: null system");
  try {
    hipStream_t st = (hipStream_t)stream;
    const HostCover& H = sys->cover->H;
    const int64_t N = H.N(), nnz = H.rowptr.back();
    if (val) PDD_HIP(hipMemcpyAsync(val, sys->val.ptr<void>(), nnz * 8, hipMemcpyDefault, st));
    if (se) PDD_HIP(hipMemcpyAsync(se, sys->se.ptr<void>(), nnz * 8, hipMemcpyDefault, st));
    if (b) PDD_HIP(hipMemcpyAsync(b, sys->b.ptr<void>(), N * 8, hipMemcpyDefault, st));
    if (se_b) PDD_HIP(hipMemcpyAsync(se_b, sys->se_b.ptr<void>(), N * 8, hipMemcpyDefault, st));
    PDD_HIP(hipStreamSynchronize(st));
    return PDD_OK;
  } catch (const HipError& e) {
    return fail(PDD_EDEVICE, e.what());
  } catch (const std::bad_alloc&) {
    return fail(PDD_ENOMEM, "pdd_system_copy: out of host memory");
  } catch (const std::exception& e) {
    return fail(PDD_EDEVICE, std::string("pdd_system_copy: ") + e.what());
  }
}

pdd_status pdd_system_csr(pdd_system sys, int64_t* rowptr, int32_t* cols, double* val, double* b, double* se,
                          void* stream) {
  if (!sys) return fail(PDD_EINVAL, "pdd_system_csr: null system");
  try {
    hipStream_t st = (hipStream_t)stream;
    const DeviceCover& D = sys->cover->D;
    const int64_t N = sys->cover->H.N(), nnz = sys->cover->H.rowptr.back();
    if (rowptr) PDD_HIP(hipMemcpyAsync(rowptr, D.rowptr.ptr<void>(), (N + 1) * 8, hipMemcpyDefault, st));
    if (cols && nnz) PDD_HIP(hipMemcpyAsync(cols, D.cols.ptr<void>(), nnz * 4, hipMemcpyDefault, st));
    if (val && nnz) PDD_HIP(hipMemcpyAsync(val, sys->val.ptr<void>(), nnz * 8, hipMemcpyDefault, st));
    if (se && nnz) PDD_HIP(hipMemcpyAsync(se, sys->se.ptr<void>(), nnz * 8, hipMemcpyDefault, st));
    if (b && N) PDD_HIP(hipMemcpyAsync(b, sys->b.ptr<void>(), N * 8, hipMemcpyDefault, st));
    PDD_HIP(hipStreamSynchronize(st));
    return PDD_OK;
  } catch (const HipError& e) {
    return fail(PDD_EDEVICE, e.what());
  } catch (const std::exception& e) {
    return fail(PDD_EDEVICE, std::string("pdd_system_csr: ") + e.what());
  }
}

pdd_status pdd_system_get_stats(pdd_system sys, pdd_system_stats* out) {
  if (!sys || !out) return fail(PDD_EINVAL, "pdd_system_get_stats: null argument");
  *out = sys->stats;
  return PDD_OK;
}

void pdd_destroy_system(pdd_system sys) { delete sys; }

}  // extern "C"
