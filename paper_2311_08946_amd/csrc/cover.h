// Host-side cover geometry (Section 2.1, eqs. 4-12) and row choice (Section 3.2).
#pragma once

#include <cstdint>
#include <string>
#include <memory>
#include <vector>

#include "pdd.h"

namespace pdd {

enum RowClass : int32_t { ROW_SPECTRAL = 0, ROW_MC = 1, ROW_BOUNDARY = 2 };

struct Bucket {
  int32_t Nr, Nt, M;
  std::vector<int32_t> fl;          // floating-list indices (position in float_ids)
};

struct HostCover {
  pdd_domain dom{};
  int32_t nc = 0;
  std::vector<double> cx, cy, r, arc0, arc1, rbf_c2;
  std::vector<int32_t> M, Nt, Nr;
  std::vector<uint8_t> floating;
  std::vector<int64_t> knot_off;    // [nc+1] stencil ranges (eq. 9)
  // knots
  std::vector<double> kx, ky, ktheta;
  std::vector<int32_t> owner, assigned, row_class;
  std::vector<uint8_t> boundary;
  // CSR pattern of C
  std::vector<int64_t> rowptr;
  std::vector<int32_t> cols;
  // floating circles
  std::vector<int32_t> float_ids;   // circle ids of floating circles
  std::vector<int32_t> float_pos;   // [nc] position in float_ids or -1
  std::vector<int64_t> node_off;    // [n_float+1]
  std::vector<int64_t> fk_off;      // [n_float+1] knots assigned to each floating circle
  std::vector<int32_t> fk_ids;
  // perimeter circles and Monte Carlo knots
  std::vector<int32_t> perim_ids;   // circle ids of perimeter circles
  std::vector<int32_t> perim_pos;   // [nc] position in perim_ids or -1
  std::vector<int32_t> mc_knots;    // knots with Monte Carlo rows, grouped by circle
  std::vector<int32_t> bnd_knots;   // boundary (junction) knots
  std::vector<Bucket> buckets;      // floating circles grouped by (Nr, Ntheta, M)
  int64_t N() const { return (int64_t)kx.size(); }
  int64_t sum_n = 0, sum_n2 = 0;
  int32_t max_n = 0, max_M = 0, max_arc = 0;
  // rule AVERAGED (eqs. 38-39): the pairs (knot i, circle m containing x_i) as
  // the rows of a second cover, each the row circle m alone gives at x_i
  // (diagonal slot included), assembled by the same kernels and then combined
  // into the rows of this cover
  std::unique_ptr<HostCover> pairs;
  std::vector<int32_t> pair_knot;   // (in `pairs`) the knot of each pair
  std::vector<int64_t> pair_seg;    // (in `pairs`) where circle m's entries start in row i of C
  std::vector<int64_t> pair_off;    // [N+1] pairs of each knot (contiguous)
  std::vector<int64_t> diag_pos;    // [N] position of C_ii in the values
};

// Returns an empty string on success, otherwise the reason the cover is invalid.
std::string build_host_cover(const pdd_domain& dom, int32_t n, const double* centres,
                             const double* radii, const int32_t* M, const int32_t* Nt,
                             const int32_t* Nr, int32_t rule, double rbf_c2, HostCover& out);

double signed_distance(const pdd_domain& dom, double x, double y);

}  // namespace pdd
