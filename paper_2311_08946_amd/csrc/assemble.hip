// pdd_assemble_G: orchestration of the floating-row kernels (per size bucket
// and chunk), the Monte Carlo path and finalisation kernels and the boundary
// rows, followed by one status read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
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

pdd_status assemble_impl(pdd_cover cover, const pdd_problem* problem, const pdd_samples* samples,
                         const pdd_mc_opts* mc, const pdd_assemble_opts* opts, hipStream_t st,
                         pdd_system* out) {
  const HostCover& H = cover->H;
  if (!H.mc_knots.empty()) {
    if (!mc) return fail(PDD_EINVAL, "pdd_assemble_G: Monte Carlo options are required");
    if (mc->paths < 2 || !(mc->h > 0.0) || mc->n_batches < 2 || mc->n_batches > 63 ||
        mc->step_cap <= 0 || mc->paths < mc->n_batches || mc->paths > ((int64_t)1 << 32))
      return fail(PDD_EINVAL, "pdd_assemble_G: bad Monte Carlo options");
    const int64_t tri = (int64_t)H.max_arc * (H.max_arc + 1) / 2;
    if ((tri + (int64_t)(mc->n_batches + 1) * H.max_arc) * (int64_t)sizeof(double) > 160 * 1024)
      return fail(PDD_EINVAL, "pdd_assemble_G: arc length and batch count exceed the 160 KiB LDS budget "
                              "of the Monte Carlo finalisation");
  }
  int dev = 0;
  PDD_HIP(hipGetDevice(&dev));
  DeviceCover& D = cover->D;
  if (!D.ready || D.device != dev) {
    D.upload(H);
    D.device = dev;
  }
  auto sys = std::make_unique<pdd_system_s>();
  sys->cover = cover;
  const int64_t N = H.N(), nnz = H.rowptr.back();
  sys->val.alloc(nnz * sizeof(double));
  sys->se.alloc(nnz * sizeof(double));
  sys->b.alloc(N * sizeof(double));
  sys->se_b.alloc(N * sizeof(double));
  PDD_HIP(hipMemsetAsync(sys->se.ptr<void>(), 0, nnz * sizeof(double), st));
  PDD_HIP(hipMemsetAsync(sys->se_b.ptr<void>(), 0, N * sizeof(double), st));

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

  // The Monte Carlo and boundary rows run on a second stream, concurrently
  // with the floating rows; both write disjoint rows of the CSR arrays.
  DevBuf lu_fail;
  lu_fail.alloc(sizeof(uint64_t) * 4);
  PDD_HIP(hipMemsetAsync(lu_fail.ptr<void>(), 0, sizeof(uint64_t) * 4, st));
  if (!D.side) PDD_HIP(hipStreamCreateWithFlags(&D.side, hipStreamNonBlocking));
  hipStream_t side = D.side;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  PDD_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
  PDD_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  } ev_guard{ev_fork, ev_join};
  PDD_HIP(hipEventRecord(ev_fork, st));
  PDD_HIP(hipStreamWaitEvent(side, ev_fork, 0));

  // ---- perimeter rows by Monte Carlo (side stream)
  const int64_t n_mc = (int64_t)H.mc_knots.size();
  const int64_t n_perim = (int64_t)H.perim_ids.size();
  DevBuf out_phi, out_g, out_steps, out_capped, gram, gram_status, hcirc;
  int32_t n_launch_mc = 0;
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
    a.n_units = n_mc * mc->n_batches;
    a.out_stride = std::max<int64_t>(1, H.max_arc);
    a.gram_stride = (int64_t)H.max_arc * (H.max_arc + 1) / 2;
    out_phi.alloc(std::max<int64_t>(1, a.n_units * a.out_stride) * sizeof(double));
    out_g.alloc(std::max<int64_t>(1, a.n_units) * sizeof(double));
    out_steps.alloc(std::max<int64_t>(1, a.n_units) * sizeof(uint64_t));
    out_capped.alloc(std::max<int64_t>(1, a.n_units) * sizeof(uint64_t));
    gram.alloc(std::max<int64_t>(1, n_perim * a.gram_stride) * sizeof(double));
    gram_status.alloc(std::max<int64_t>(1, n_perim) * sizeof(int32_t));
    a.out_phi = out_phi.ptr<double>();
    a.out_g = out_g.ptr<double>();
    a.out_steps = out_steps.ptr<uint64_t>();
    a.out_capped = out_capped.ptr<uint64_t>();
    launch_mc_paths(P, dp.const_coef != 0, a, side);
    launch_gram_cholesky(a, (int32_t)n_perim, gram.ptr<double>(), gram_status.ptr<int32_t>(), side);
    launch_mc_finalize(a, (int32_t)n_mc, H.max_arc, gram.ptr<double>(), sys->val.ptr<double>(),
                       sys->se.ptr<double>(), sys->b.ptr<double>(), sys->se_b.ptr<double>(), side);
    PDD_HIP(hipGetLastError());
    hipLaunchKernelGGL(reduce_u64_kernel, dim3(1), dim3(256), 0, side, out_steps.ptr<uint64_t>(),
                       a.n_units, lu_fail.ptr<uint64_t>() + 1);
    hipLaunchKernelGGL(reduce_u64_kernel, dim3(1), dim3(256), 0, side, out_capped.ptr<uint64_t>(),
                       a.n_units, lu_fail.ptr<uint64_t>() + 2);
    if (n_perim > 0)
      hipLaunchKernelGGL(reduce_i32_kernel, dim3(1), dim3(256), 0, side, gram_status.ptr<int32_t>(),
                         n_perim, lu_fail.ptr<uint64_t>() + 3);
    n_launch_mc = 3;
    timer.end(e);
  }
  launch_boundary_rows(P, D.bnd_knots.ptr<int32_t>(), (int32_t)H.bnd_knots.size(), D.kx.ptr<double>(),
                       D.ky.ptr<double>(), D.rowptr.ptr<int64_t>(), sys->val.ptr<double>(),
                       sys->se.ptr<double>(), sys->b.ptr<double>(), sys->se_b.ptr<double>(), side);
  PDD_HIP(hipGetLastError());
  PDD_HIP(hipEventRecord(ev_join, side));

  // ---- floating rows, bucket by bucket, in chunks that fit the budget.  The
  //      factors are kept when asked for and when all of them fit; otherwise
  //      one chunk buffer per bucket is reused (stream order protects it).
  int32_t n_launch_spectral = 0;
  LuScratch lu_work;
  int64_t kept = 0;
  for (size_t bi = 0; bi < D.buckets.size(); ++bi) {
    BucketData& bk = *D.buckets[bi];
    const int64_t per = factor_bytes_per_circle(bk);
    const int32_t chunk = keep_all ? bk.count
                                   : (int32_t)std::min<int64_t>(bk.count, std::max<int64_t>(1, budget / per));
    std::unique_ptr<BucketFactors> reuse;
    for (int32_t first = 0; first < bk.count; first += chunk) {
      const int32_t cnt = std::min(chunk, bk.count - first);
      std::unique_ptr<BucketFactors> f;
      if (keep_all || !reuse) {
        f = std::make_unique<BucketFactors>();
        f->bucket = (int32_t)bi;
        alloc_factors(*f, bk, keep_all ? cnt : chunk);
      } else {
        f = std::move(reuse);
      }
      n_launch_spectral += factor_chunk(D, bk, S, plan, *f, first, cnt, lu_work, st, &timer,
                                        sys->val.ptr<double>(), sys->b.ptr<double>());
      hipLaunchKernelGGL(reduce_i32_kernel, dim3(1), dim3(256), 0, st, f->status.ptr<int32_t>(),
                         (int64_t)cnt, lu_fail.ptr<uint64_t>());
      if (keep_all) {
        kept += (int64_t)cnt * per;
        sys->factors.push_back(std::move(f));
      } else {
        reuse = std::move(f);
      }
    }
    if (reuse) PDD_HIP(hipStreamSynchronize(st));   // before its buffers are freed
  }

  PDD_HIP(hipStreamWaitEvent(st, ev_join, 0));
  timer.end(t_all);

  uint64_t flags[4] = {0, 0, 0, 0};
  PDD_HIP(hipMemcpyAsync(flags, lu_fail.ptr<void>(), sizeof(flags), hipMemcpyDeviceToHost, st));
  PDD_HIP(hipStreamSynchronize(st));
  pdd_system_stats& s = sys->stats;
  s.path_steps = (int64_t)flags[1];
  s.capped_paths = (int64_t)flags[2];
  s.paths = mc ? n_mc * mc->paths : 0;
  s.breakdowns = (int32_t)(flags[0] + flags[3]);
  s.n_launch_spectral = n_launch_spectral;
  s.factor_bytes = kept;
  s.recompute = sys->recompute ? 1 : 0;
  s.n_launch_mc = n_launch_mc;
  s.ms_sample = timer.total(PH_SAMPLE);
  s.ms_build = timer.total(PH_BUILD);
  s.ms_lu = timer.total(PH_LU);
  s.ms_solve = timer.total(PH_SOLVE);
  s.ms_eval = timer.total(PH_EVAL);
  s.ms_mc = timer.total(PH_MC);
  s.ms_total = timer.total(PH_TOTAL);
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
  }
}

pdd_status pdd_system_get_stats(pdd_system sys, pdd_system_stats* out) {
  if (!sys || !out) return fail(PDD_EINVAL, "pdd_system_get_stats: null argument");
  *out = sys->stats;
  return PDD_OK;
}

void pdd_destroy_system(pdd_system sys) { delete sys; }

}  // extern "C"
