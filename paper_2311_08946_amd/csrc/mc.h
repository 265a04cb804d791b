// Monte Carlo (perimeter rows) and boundary-row launchers (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "device_common.h"

namespace pdd {

struct McArgs {
  // cover tables (device)
  const int32_t* mc_knots;     // [n_mc] knots with Monte Carlo rows
  const int32_t* assigned;     // [N]
  const int32_t* perim_ids;    // [n_perim]
  const int32_t* perim_pos;    // [n_circles]
  const double* cx;
  const double* cy;
  const double* rad;
  const double* arc0;
  const double* arc1;
  const double* rbf_c2;
  const int64_t* knot_off;
  const double* kx;
  const double* ky;
  const double* ktheta;
  const int64_t* rowptr;
  const double* h_circle;      // [n_circles] or null
  // options
  double h;
  uint64_t seed;
  int64_t paths;
  int32_t n_batches;
  int32_t step_cap;
  int32_t scheme;              // 0 plain Euler, 1 boundary-shifted (Gobet-Menozzi)
  int64_t n_units;             // n_mc * n_batches
  // per-unit results (device)
  double* out_phi;             // [n_units][out_stride]
  int64_t out_stride;
  double* out_g;               // [n_units]
  uint64_t* out_steps;
  uint64_t* out_capped;
  uint64_t* out_gamma;         // [n_units] paths that exited on Gamma_m
  int64_t gram_stride;         // max_arc^2
};

// `host`: the host copy of *P (selects the kernel variant).
void launch_mc_paths(const DevProblem* P, const DevProblem& host, const McArgs& a, hipStream_t st);
void launch_gram_cholesky(const McArgs& a, int32_t n_perim, double* Lf, int32_t* status,
                          hipStream_t st);
void launch_mc_finalize(const McArgs& a, int32_t n_mc, int32_t max_arc, const double* Lf,
                        double* val, double* se, double* b, double* se_b, hipStream_t st);
void launch_boundary_rows(const DevProblem* P, const int32_t* ids, int32_t count,
                          const double* kx, const double* ky, const int64_t* rowptr, double* val,
                          double* se, double* b, double* se_b, hipStream_t st);

}  // namespace pdd
