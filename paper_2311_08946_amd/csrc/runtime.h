// Device memory ownership, per-cover device tables and the opaque handles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "cover.h"
#include "device_common.h"
#include "kernels.h"

namespace pdd {

pdd_status fail(pdd_status code, const std::string& msg);

struct HipError : std::runtime_error {
  hipError_t code;
  HipError(hipError_t c, const std::string& where)
      : std::runtime_error(where + ": " + hipGetErrorString(c)), code(c) {}
};

#define PDD_HIP(call)                                                   \
  do {                                                                  \
    hipError_t e_ = (call);                                             \
    if (e_ != hipSuccess) throw ::pdd::HipError(e_, #call);             \
  } while (0)

// Device memory of the library.  Blocks of at least kCacheMinBytes return to a
// per-device cache when released and are handed out again for the same
// rounded size, so repeated assemblies of one problem (factors, values, work
// areas: tens of GB) do not go through hipMalloc / hipFree every time -- the
// runtime's release of such blocks slows down by orders of magnitude after a
// few cycles.  A released block is cached only after its device is
// synchronised (the guarantee hipFree gives), the cache holds at most half of
// the device's memory, and a failed allocation empties it and retries.
constexpr size_t kCacheMinBytes = size_t(4) << 20;
void* device_alloc(size_t bytes, int& device);          // throws HipError
void device_free(void* p, size_t bytes, int device);
size_t device_cache_release();                          // frees every cached block; returns bytes

// Owning device allocation.
class DevBuf {
 public:
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p_) device_free(p_, bytes_, dev_);
    p_ = nullptr;
    bytes_ = 0;
  }
  void alloc(size_t bytes) {
    release();
    if (bytes == 0) return;
    p_ = device_alloc(bytes, dev_);
    bytes_ = bytes;
  }
  template <class T>
  void upload(const std::vector<T>& v) {
    alloc(v.size() * sizeof(T));
    if (!v.empty()) PDD_HIP(hipMemcpy(p_, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  }
  template <class T>
  T* ptr() const { return static_cast<T*>(p_); }
  size_t bytes() const { return bytes_; }

 private:
  void* p_ = nullptr;
  size_t bytes_ = 0;
  int dev_ = -1;
};

struct BucketData {
  int32_t Nr = 0, Nt = 0, M = 0, Nc = 0, n = 0, ld = 0, nrhs = 0, count = 0;
  DevBuf tables;               // operator tables
  DevBuf fl;                   // [count] floating-list indices
  BucketTables T{};
  std::vector<double> host_H;
  void build(int Nr, int Nt, int M);
};

struct DeviceCover {
  bool ready = false;
  int device = -1;
  hipStream_t side = nullptr;           // second stream for the Monte Carlo rows
  ~DeviceCover() { if (side) (void)hipStreamDestroy(side); }
  DevBuf cx, cy, rad, arc0, arc1, rbf_c2, kx, ky, ktheta;
  DevBuf knot_off, rowptr, cols, assigned, float_ids, node_off, fk_off, fk_ids;
  DevBuf perim_ids, perim_pos, mc_knots, bnd_knots;
  DevBuf pair_off, diag_pos, pair_knot, pair_seg;   // rule AVERAGED (see HostCover)
  DevBuf rt_rowptr, rt_cols, rt_perm;   // transpose pattern of C (built on first use)
  bool have_transpose = false;
  // Circle-blocked structure of C (built on the first solve; rules with one
  // subdomain per row): row i holds C_ii and the stencil of its circle, a
  // contiguous knot range starting at blk_so[i]; blk_circ_rows lists the rows
  // of each circle (offsets blk_circ_off), which are the only rows whose
  // stencils hold that circle's knots.
  DevBuf blk_so, blk_circ_off, blk_circ_rows, blk_circ_roff;   // blk_circ_roff: rowptr[i] - i per slot
  bool have_blocked = false;
  bool blocked_ok = false;
  bool tuned = false;                   // schedule chosen by the autotuner for this cover
  bool tuned_mixed = true;
  int tuned_cap = 0;
  bool tuned_lookahead = true;
  // the last autotuned assembly's Monte Carlo and floating-row times (ms)
  float last_ms_mc = 0.0f, last_ms_float = 0.0f;
  std::vector<std::unique_ptr<BucketData>> buckets;
  void upload(const HostCover& H);
  ChunkDesc chunk(const BucketData& b, int32_t first, int32_t count) const;
};

pdd_status make_dev_problem(const pdd_problem& p, DevProblem& D);

// Factor storage of one bucket, kept for the adjoint.
struct BucketFactors {
  int32_t bucket = -1;
  int32_t first = 0, count = 0;
  int64_t stride = 0;          // doubles per matrix
  DevBuf A;                    // [count][n][ld]  LU factors and W
  DevBuf piv;                  // [count][n]
  DevBuf rowscale;             // [count][n]
  DevBuf status;               // [count]
};

// A batch of matrices (any mix of sizes) and its work lists: for each launch
// kind and step, a prefix array over the matrices of their work units.
struct LuPlan {
  std::vector<LuItem> items;
  int32_t count = 0;
  int nsteps = 0;
  std::vector<int32_t> pre;      // [kind][step][count + 1]
  std::vector<int32_t> totals;   // [kind][step]
  std::vector<int32_t> own_threads;   // [class 0, 1][step]: block size of the row-ownership panels
  bool wide_rhs = false;              // some matrix has more than 128 right-hand sides
  DevBuf d_items, d_pre;
  // the second stream of the look-ahead and its per-step events
  hipStream_t side = nullptr;
  std::vector<hipEvent_t> ev_main, ev_rest;
  LuPlan() = default;
  LuPlan(const LuPlan&) = delete;
  LuPlan& operator=(const LuPlan&) = delete;
  ~LuPlan();
  void build(const std::vector<LuItem>& its);
  // Issues the launch sequence on st (with lookahead, also on the plan's
  // second stream, joined back into st before the back substitution);
  // grid_cap bounds the workgroups of the tiled launches (each workgroup
  // strides over the list).  Returns launches.
  int launch(hipStream_t st, int grid_cap, bool lookahead = true) const;
};

// Device bytes of one circle's factors in a bucket (matrix, pivots, row
// scales, status).
inline int64_t factor_bytes_per_circle(const BucketData& bk) {
  return (int64_t)bk.n * bk.ld * 8 + (int64_t)bk.n * (4 + 8) + 4;
}

// Phase timing hooks of the orchestration (events on the given stream).
enum { PH_SAMPLE, PH_BUILD, PH_LU, PH_SOLVE, PH_EVAL, PH_MC, PH_TOTAL };
struct PhaseHooks {
  virtual int begin(int phase, hipStream_t s = nullptr) = 0;
  virtual void end(int idx) = 0;
  virtual ~PhaseHooks() = default;
};

// Growable device work area of the LU launches.
struct LuScratch {
  DevBuf buf;
  size_t bytes = 0;
};

void alloc_factors(BucketFactors& f, const BucketData& bk, int32_t count);

// Builds, factorises and solves circles [first, first + cnt) of bucket bk into
// f (allocated for at least cnt circles); with val/b non-null also
// interpolates and scatters their rows.  hooks may be null.  Returns the
// number of kernel launches.
int factor_chunk(const DeviceCover& D, const BucketData& bk, const NodeSamples& S, int plan,
                 BucketFactors& f, int32_t first, int32_t cnt, LuScratch& ws, hipStream_t st,
                 PhaseHooks* hooks, double* val, double* b);

}  // namespace pdd

namespace pdd {
// BiCGStab scratch (device vectors and partial sums, two pinned convergence
// records), kept by the cover between solves so that a solve on a new system
// allocates nothing; concurrent solves each take their own.
struct SolveScratch {
  int device = -1;
  DevBuf work;
  double* pinned = nullptr;
  ~SolveScratch() { if (pinned) (void)hipHostFree(pinned); }
};
}  // namespace pdd

struct pdd_cover_s {
  pdd::HostCover H;
  pdd::DeviceCover D;
  pdd::DeviceCover DP;   // rule AVERAGED: the pair rows (H.pairs)
  std::mutex solve_mu;
  std::vector<std::unique_ptr<pdd::SolveScratch>> solve_free;
};

struct pdd_system_s {
  pdd_cover cover = nullptr;
  pdd::DevBuf val, b, se, se_b;
  pdd::DevBuf problem;               // DevProblem
  pdd::DevBuf samples;               // [7][sum_n] node samples (owned copy)
  std::vector<std::unique_ptr<pdd::BucketFactors>> factors;
  bool recompute = false;            // factors exceed the budget: backward rebuilds them by chunks
  int64_t budget = 0;                // device bytes allowed for factors
  int32_t plan = 0;
  pdd_system_stats stats{};
  std::vector<double> host_problem_bytes;
  pdd::DevBuf val_t;                   // C^T values (formed on the first transposed solve)
  pdd::DevBuf vblk, dg;                // circle-blocked values: per row its stencil entries
                                       // (at rowptr[i] - i) and the diagonal (formed on the first solve)
  bool have_vblk = false;
};
