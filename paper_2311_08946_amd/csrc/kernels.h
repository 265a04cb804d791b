// Launch wrappers of the HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "device_common.h"

namespace pdd {

// Per-size tables of one bucket (Nr, Ntheta, M) of floating circles, on the device.
struct BucketTables {
  int32_t Nr, Nt, M, Nc;       // Nc = 2 Nr + 1 (radial grid x_0..x_Nc)
  int32_t n, ld, nrhs;         // n = Nr Nt, ld = n + rhs_pad, nrhs = M + 1
  const double* Dr;            // [Nr][Nc+1]  rows 1..Nr of the Chebyshev matrix
  const double* D2r;           // [Nr][Nc+1]  rows 1..Nr of its square
  const double* d1t;           // [Nt] first Fourier derivative by index difference
  const double* d2t;           // [Nt] second Fourier derivative by index difference
  const double* H;             // [Nt][M] M-knot cardinal functions at the ring angles
  const double* xr;            // [Nc+1] Chebyshev points
  const double* bw;            // [Nc+1] barycentric weights
  const double* cs;            // [Nt] cos theta_l
  const double* sn;            // [Nt] sin theta_l
};

// Per-chunk description of the floating circles being processed.
struct ChunkDesc {
  int32_t count;               // circles in this chunk
  const int32_t* fl;           // [count] floating-list index of each circle
  const int32_t* float_ids;    // [n_float] circle id
  const double* cx;            // [n_circles]
  const double* cy;
  const double* rad;
  const int64_t* node_off;     // [n_float+1]
  const int64_t* fk_off;       // [n_float+1]
  const int32_t* fk_ids;       // knots assigned to floating circles
  const int64_t* knot_off;     // [n_circles+1]
  const double* kx;            // [N]
  const double* ky;
  const int64_t* rowptr;       // [N+1]
};

struct NodeSamples {
  const double* s[7];          // axx, axy, ayy, bx, by, c, f  [sum_n]
};

// K1: augmented, row-equilibrated collocation rows [A_II | A_IB H | -F | 0].
void launch_colloc_build(const BucketTables& T, const ChunkDesc& C, const NodeSamples& S,
                         double* A, int64_t mat_stride, double* rowscale, hipStream_t st);
// K2/K3: in-place LU with partial pivoting of the n x n block, applied to all ld
// columns (forward elimination of the right-hand sides), then back
// substitution U W = R' on the right-hand-side columns.
struct LuWork;                 // per-matrix step data (device)
struct LuItem {                // one matrix of a batch (device pointers)
  double* A;                   // [n][ld]
  int32_t* piv;                // [n]
  int32_t* status;             // 1 = zero pivot met
  LuWork* work;                // lu_work_bytes_per_matrix(n) bytes: LuWork, then
  double* uinv;                //   the inverses of U's 32 x 32 diagonal blocks
  int32_t n, ld, nrhs, cls;    // cls = lu_panel_class(n)
};
// launch kinds: the panel kernel per size class, then the tiled kinds (the
// U-row tiles split into the first tile of each matrix and the rest)
enum {
  LU_PUPD, LU_PANEL0, LU_PANEL1, LU_PANEL2, LU_PANEL3, LU_LSWAP, LU_UROW0, LU_UREST, LU_BDIAG, LU_BUPD, LU_KINDS
};
int lu_panel_class(int n);
size_t lu_work_bytes_per_matrix(int32_t n);
size_t lu_work_header_bytes();   // sizeof(LuWork): the inverses of U's blocks follow
size_t lu_workspace_bytes(int32_t count, int32_t n);
// Work units of one matrix in one launch of the given kind at the given step.
int lu_plan_tiles(const LuItem& it, int kind, int step);
// One bucket chunk of `count` matrices with a contiguous work area; returns
// the number of kernel launches.
int launch_lu_solve(const BucketTables& T, int32_t count, double* A, int64_t mat_stride,
                    int32_t* piv, int32_t* status, void* work, hipStream_t st);
// K4: interpolation at the assigned knots and scatter into CSR values and r.
void launch_eval_scatter(const BucketTables& T, const ChunkDesc& C, const double* A,
                         int64_t mat_stride, double* val, double* b, hipStream_t st);
// Node sampling of the problem's fields.
void launch_sample_nodes(const DevProblem* P, const BucketTables& T, const ChunkDesc& C,
                         double* const out[7], hipStream_t st);

}  // namespace pdd
