/*
 * pdd.h -- C ABI of the MI355X (gfx950) library that assembles and solves the
 * explicit interfacial system  C u = r  of the overlapping-circle stochastic
 * substructuring method (Moron-Vidal, Bernal, Suzuki, arXiv 2311.08946).
 *
 * Problem (Section 2, eqs. 1-3):  L u + c u + f = 0 in Omega, u = g on the
 * boundary, with L = a_xx/2 d_xx + a_xy d_xy + a_yy/2 d_yy + b_x d_x + b_y d_y
 * and c <= 0.  Omega is covered by open disks (eqs. 4-8); the unknowns are the
 * solution values at N knots on the circles (eqs. 9-12).  Row i of C (eqs.
 * 28-30) comes from one subdomain containing knot i (Section 3.2):
 *   - floating circle: C_ij = G_j(x_i), r_i = B(x_i) from local problems (eqs.
 *     31-35) solved by polar Chebyshev x Fourier collocation (Section 3.3,
 *     eqs. 40-41) -- batched dense LU on the GPU;
 *   - perimeter subdomain: Monte Carlo of the Feynman-Kac expectations (eqs.
 *     29-30 with the SDE of eq. 53), plain Euler-Maruyama on Philox4x32-10
 *     streams, interface data interpolated by inverse multiquadrics (eqs.
 *     19-22);
 *   - junction knot on the boundary: C_ii = 1, r_i = g(x_i).
 *
 * Conventions shared by every entry point:
 *   - Every function returns a pdd_status; PDD_OK is 0.  On error a message
 *     is available from pdd_last_error() (thread-local, valid until the next
 *     call on the same thread).  No C++ exception crosses this boundary.
 *   - Handles (pdd_cover, pdd_system) are opaque and owned by the library;
 *     release them with pdd_destroy_cover / pdd_destroy_system.
 *   - Array arguments are owned by the caller and only read (or written, for
 *     outputs) during the call.  "host" arrays are ordinary CPU memory;
 *     "device" arrays are HIP device memory on the current device.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Device work is
 *     stream-ordered; functions that must report a device-side status (pivot
 *     breakdown, path-step cap, solver convergence) synchronise that stream
 *     before returning.
 *   - All floating point is IEEE binary64.
 *   - Calls that take the same cover or system handle must not overlap, with
 *     two exceptions: pdd_solve_G calls on one system may run concurrently
 *     (each takes its own work area; forming C^T is locked), and read-only
 *     queries (info, knots, pattern, nodes, stats) may run at any time.
 */
#ifndef PDD_H
#define PDD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pdd_status;
enum {
  PDD_OK = 0,
  PDD_EINVAL = 1,      /* bad argument (null pointer, size out of range)          */
  PDD_ECOVER = 2,      /* cover violates eq. 5, an uncovered knot, multi-arc Gamma */
  PDD_ENOMEM = 3,      /* device or host allocation failed                         */
  PDD_EDEVICE = 4,     /* HIP runtime error                                        */
  PDD_ENOCONV = 5,     /* iterative solve did not reach the tolerance              */
  PDD_EPATHCAP = 6,    /* a Monte Carlo path exceeded the step cap                 */
  PDD_EBREAKDOWN = 7   /* zero pivot in a collocation LU or a non-SPD RBF Gram     */
};

typedef struct pdd_cover_s* pdd_cover;
typedef struct pdd_system_s* pdd_system;

const char* pdd_last_error(void);

/*
 * Device memory.  Blocks of 4 MiB and more that the library releases (when a
 * system is destroyed, or at the end of a call that used work areas) are kept
 * in a per-device cache and reused by later calls of the same sizes, instead
 * of going back to the HIP runtime: repeated assemblies of one problem then
 * allocate nothing new.  A block enters the cache only after its device has
 * been synchronised; the cache holds at most half of the device's memory; an
 * allocation that fails empties it and tries again.
 * pdd_release_cached_memory frees every cached block (all devices) and
 * returns the number of bytes freed.  No compute happens here.
 */
int64_t pdd_release_cached_memory(void);

/* ---------------------------------------------------------------- problem */

enum { PDD_DOMAIN_BOX = 0, PDD_DOMAIN_DISK = 1 };
#define PDD_MAX_HOLES 4

/* Omega: the open box (x0,x1)x(y0,y1), or the open disk |x-c| < R minus up to
 * four closed disks (hx, hy, hr). */
typedef struct pdd_domain {
  int32_t kind;
  int32_t n_holes;
  double x0, x1, y0, y1;
  double cx, cy, R;
  double holes[PDD_MAX_HOLES][3];
} pdd_domain;

enum {
  PDD_FIELD_CONST = 0,     /* value = base                                            */
  PDD_FIELD_SINSUM = 1,    /* base + sum_q a_q sin(2 pi (b_q x + c_q y) + d_q),
                              then min(., 0) if clip_nonpos                           */
  PDD_FIELD_CPOLY_RE = 2,  /* Re sum_k (a_k + i b_k) (x + i y)^k, k < n_terms        */
  PDD_FIELD_DERIVED_F = 3, /* f = -(L u + c u) for the problem's manufactured u      */
  PDD_FIELD_EQ46 = 4       /* the manufactured solution of Section 4 (eq. 46), no
                              parameters: 3 + sin(sqrt(1 + x^2/100 + y^2/50))/3
                              + tanh(sin(3x/25 + y/20) + sin(x/20 - 3y/25))/3       */
};
#define PDD_MAX_TERMS 16

/* A coefficient field, evaluated on the device at nodes and along paths.
 * The term arrays are host pointers read during the call that receives them. */
typedef struct pdd_field {
  int32_t kind;
  int32_t n_terms;         /* <= PDD_MAX_TERMS                                       */
  int32_t clip_nonpos;
  int32_t reserved;
  double base;
  const double* a;
  const double* b;
  const double* c;
  const double* d;
} pdd_field;

/* The model problem of eq. 1.  `u` is the manufactured solution used by
 * PDD_FIELD_DERIVED_F (SINSUM, CPOLY_RE or EQ46); otherwise it is ignored. */
typedef struct pdd_problem {
  pdd_domain domain;
  pdd_field axx, axy, ayy, bx, by, c, f, g, u;
} pdd_problem;

enum {
  PDD_WHICH_AXX = 0, PDD_WHICH_AXY = 1, PDD_WHICH_AYY = 2, PDD_WHICH_BX = 3, PDD_WHICH_BY = 4,
  PDD_WHICH_C = 5, PDD_WHICH_F = 6, PDD_WHICH_G = 7, PDD_WHICH_U = 8
};

/*
 * pdd_eval_field -- evaluates one field of the problem (eq. 1: a coefficient,
 * the source f, the boundary data g, or the manufactured solution u) at n
 * points on the device.
 *   xy   device [2n] interleaved (x, y);  out  device [n]
 * Errors: PDD_EINVAL (bad field or `which`), PDD_EDEVICE.  Stream-ordered.
 */
pdd_status pdd_eval_field(const pdd_problem* problem, int32_t which, const double* xy, int64_t n,
                          double* out, void* stream);

/* ------------------------------------------------------------------ cover */

/* Row choice: the deepest floating circle containing the knot (else the deepest
 * perimeter one); the deepest of any kind; or (AVERAGED, eqs. 38-39) the sum of
 * the expectations of every containing circle, C_ii = their number. */
enum { PDD_RULE_FLOAT_FIRST_MAX_DEPTH = 0, PDD_RULE_MAX_DEPTH = 1, PDD_RULE_AVERAGED = 2 };

typedef struct pdd_cover_opts {
  int32_t rule;            /* row choice of Section 3.2 (see pdd_build_cover)         */
  int32_t reserved;
  double rbf_c2;           /* IMQ shape c^2 of eq. 19; <= 0: 1.5 (44/M)^2 per circle   */
} pdd_cover_opts;

/*
 * pdd_build_cover -- geometry of Section 2.1 (eqs. 4-12) and the row choice of
 * Section 3.2, computed on the host.
 *   centres  host [2*n_circles], (x, y) per circle
 *   radii    host [n_circles]
 *   M        host [n_circles]  knots per full circle (even)
 *   Ntheta   host [n_circles]  angular collocation nodes (even)
 *   Nr       host [n_circles]  interior radial collocation nodes (>= 1)
 * Circle m is floating if its closed disk lies in Omega; otherwise its
 * interface must be a single arc of the circle inside closure(Omega).
 * Floating knots: angles 2 pi j / M.  Arc knots: the same angles inside the
 * arc (keeping dtheta/4 away from its ends) plus one junction knot at each
 * end.  Knots are numbered circle by circle in increasing local angle.  Row
 * rule FLOAT_FIRST_MAX_DEPTH: the deepest floating circle strictly containing
 * the knot, else the deepest perimeter one; MAX_DEPTH: the deepest of all;
 * AVERAGED (eqs. 38-39): every circle strictly containing the knot, each
 * contributing its own row (the pairs (knot, circle) are numbered knot-major,
 * circles by index); row_class and assigned of pdd_cover_knots still report
 * the FLOAT_FIRST_MAX_DEPTH choice.
 * Errors: PDD_EINVAL (also an unknown rule), PDD_ECOVER (uncovered knot,
 * multi-arc interface, circle outside Omega), PDD_ENOMEM.  No device work is
 * done.
 */
pdd_status pdd_build_cover(const pdd_domain* domain, int32_t n_circles,
                           const double* centres, const double* radii,
                           const int32_t* M, const int32_t* Ntheta, const int32_t* Nr,
                           const pdd_cover_opts* opts, pdd_cover* out);

typedef struct pdd_cover_info {
  int64_t N;               /* knots = unknowns                                       */
  int64_t nnz;             /* entries of C                                           */
  int64_t n_circles, n_float, n_perim;
  int64_t n_spectral_rows, n_mc_rows, n_boundary_rows;
  int64_t sum_n;           /* collocation nodes over floating circles                */
  int64_t sum_n2;          /* sum of n^2 over floating circles                       */
  int32_t max_n, max_M, max_arc, n_buckets;
} pdd_cover_info;

/* Sizes of the cover (Section 2.1, eqs. 9-12: knots, stencils, rows by kind;
 * Section 3.3: collocation sizes).  Host only. */
pdd_status pdd_cover_get_info(pdd_cover cover, pdd_cover_info* out);

/* Knot table of eqs. 9-12 and the row choice of Section 3.2 (host outputs,
 * any may be NULL): xy [2N]; row_class [N]
 * (0 spectral, 1 Monte Carlo, 2 boundary); assigned [N] (circle of the row,
 * -1 for boundary rows); owner [N] (circle the knot lies on). */
pdd_status pdd_cover_knots(pdd_cover cover, double* xy, int32_t* row_class,
                           int32_t* assigned, int32_t* owner);

/* CSR pattern of C (eqs. 28-30; host outputs): rowptr [N+1], cols [nnz]; columns of each
 * row increase; row i holds i and, unless boundary, the stencil of its circle
 * (of every containing circle under rule AVERAGED). */
pdd_status pdd_cover_pattern(pdd_cover cover, int64_t* rowptr, int32_t* cols);

/* Collocation nodes of the floating circles (Section 3.3, eq. 40; host outputs): xy [2*sum_n],
 * circle-major, node q = (j-1) Ntheta + l at radius r cos(j pi/(2 Nr + 1)) and
 * angle 2 pi l / Ntheta; node_off [n_float+1]; float_ids [n_float]. */
pdd_status pdd_cover_nodes(pdd_cover cover, double* xy, int64_t* node_off, int32_t* float_ids);

void pdd_destroy_cover(pdd_cover cover);

/* -------------------------------------------------------------- assemble */

/* Node samples of the seven coefficients of eq. 1 at the collocation nodes of
 * the floating circles (device [sum_n] each, layout of pdd_cover_nodes).  A
 * NULL member is sampled from the problem's field on the device. */
typedef struct pdd_samples {
  const double *axx, *axy, *ayy, *bx, *by, *c, *f;
} pdd_samples;

typedef struct pdd_mc_opts {
  int64_t paths;           /* Ntilde paths per perimeter knot                         */
  double h;                /* Euler step                                              */
  uint64_t seed;           /* Philox key = (seed mod 2^32, seed div 2^32)              */
  int32_t n_batches;       /* batches for standard errors (2..63)                      */
  int32_t step_cap;        /* maximum steps of one path (> 0)                          */
  const double* h_per_circle;  /* host [n_circles] or NULL: per-circle step            */
  int32_t scheme;          /* PDD_MC_EULER or PDD_MC_SHIFTED (see pdd_assemble_G)      */
  int32_t reserved;
} pdd_mc_opts;

enum { PDD_MC_EULER = 0, PDD_MC_SHIFTED = 1 };

enum { PDD_PLAN_BATCHED = 0, PDD_PLAN_PER_CIRCLE = 1, PDD_PLAN_AUTOTUNED = 2 };

/*
 * Schedule of the floating circles (batching of the size buckets, not in the
 * paper).  Circles are grouped in size buckets (Nr, Ntheta, M); a group is a
 * set of circles whose factors are resident together (at most
 * hbm_budget_bytes).  Each group goes through one build launch per bucket,
 * one sequence of persistent LU launches over all its matrices whatever their
 * size (per 128-column step: panel, U-row and trailing-update launches; then
 * the back substitution), and one evaluation launch per bucket.
 *   PDD_PLAN_BATCHED    groups as given by mixed_buckets / grid_cap / use_graph /
 *                       no_lookahead;
 *   PDD_PLAN_PER_CIRCLE the plain loop: one circle per group;
 *   PDD_PLAN_AUTOTUNED  the library times the candidate schedules on a sample
 *                       of each bucket on first use with a cover and keeps the
 *                       fastest for that cover (stats report the choice).
 */
typedef struct pdd_assemble_opts {
  int32_t plan;            /* PDD_PLAN_BATCHED, PDD_PLAN_PER_CIRCLE or PDD_PLAN_AUTOTUNED */
  int32_t keep_factors;    /* keep LU factors for pdd_assemble_G_backward              */
  int64_t hbm_budget_bytes;/* device bytes allowed for factor storage; 0 = 64 GiB.
                              Assembly processes each size bucket in chunks of at most
                              this many bytes of factors.  With keep_factors, the
                              factors are kept when all of them fit; otherwise the
                              system keeps a copy of the node samples and
                              pdd_assemble_G_backward recomputes the factors chunk by
                              chunk (stats.recompute = 1)                              */
  int32_t mixed_buckets;   /* 1: every group takes the same share of every bucket (one
                              LU launch sequence serves all sizes); 0: groups hold one
                              bucket each                                             */
  int32_t grid_cap;        /* workgroups of the tiled LU launches, as a multiple of the
                              compute units (each strides over its work list);
                              0 = one workgroup per tile                              */
  int32_t use_graph;       /* 1: capture the LU launch sequence of a group in a HIP
                              graph and replay it for groups of the same shape; only
                              when such groups follow (transient factor buffers and
                              more than one group), otherwise launched directly      */
  int32_t no_lookahead;    /* 0: the U-row tiles right of the next panel run on a
                              second stream beside the next step's panel
                              (look-ahead); 1: every LU launch in order on one
                              stream                                                  */
  int32_t mc_order;        /* Monte Carlo rows against the floating rows: 0 = beside
                              them, except that PDD_PLAN_AUTOTUNED starts them after
                              the floating rows when the last assembly on the cover
                              found them at least 0.8 times as long; 1 = always
                              beside; 2 = always after.  The results are the same.  */
  int32_t reserved;
} pdd_assemble_opts;

/*
 * pdd_assemble_G -- builds C (CSR values on the pdd_cover_pattern layout), r,
 * and per-entry Monte Carlo standard errors.  Floating rows: for each floating
 * circle the collocation matrix [A_II | A_IB] of eq. 40 is built from the node
 * samples, LU-factorised with partial pivoting together with the right-hand
 * sides [A_IB H | -F] (eqs. 32, 35, 41), and the solutions are interpolated at
 * the knots assigned to the circle.  Perimeter rows: `mc->paths` Euler paths
 * per knot; step k of path p from knot i draws Philox4x32-10 at counter
 * (k, p, i, 0).  Scheme PDD_MC_SHIFTED is the boundary-shifted Euler scheme of
 * Gobet and Menozzi (the paper's ref. [15]): an end point inside the
 * subdomain closer to a boundary piece (the circle, a box side, the disk's
 * outer circle or a hole) than c0 sqrt(h) |sigma^T n| (n the piece's normal,
 * sigma the Cholesky factor of a at the step's start, c0 = -zeta(1/2) /
 * sqrt(2 pi)) stops the path after that step, at its projection onto the
 * nearest such piece; end points outside exit at the first crossing as in
 * PDD_MC_EULER.  Boundary rows: C_ii = 1, r_i = g(x_i).  Rule AVERAGED: each
 * pair (knot i, circle m) is assembled as the row circle m gives at x_i (the
 * pair's index takes the place of i in the Philox counter), then row i is
 * C_ii = number of pairs, the pairs' stencil entries, r_i = sum of the
 * pairs' r in pair order, standard error of r_i their quadrature sum.
 *   samples  may be NULL (all sampled on the device)
 *   out      receives a system handle owning the device results
 * Errors: PDD_EINVAL, PDD_ENOMEM, PDD_EDEVICE, PDD_EBREAKDOWN, PDD_EPATHCAP.
 * Synchronises `stream` once at the end to read the device status.
 */
pdd_status pdd_assemble_G(pdd_cover cover, const pdd_problem* problem,
                          const pdd_samples* samples, const pdd_mc_opts* mc,
                          const pdd_assemble_opts* opts, void* stream, pdd_system* out);

/* Copies the assembled C and r of eqs. 28-30 to caller buffers (device or
 * host, any may be NULL): val [nnz] on the pdd_cover_pattern layout, b [N]
 * (= r), se [nnz] (Monte Carlo standard error of each entry, 0 if exact),
 * se_b [N].  Enqueued on `stream`, which is synchronised before returning. */
pdd_status pdd_system_copy(pdd_system sys, double* val, double* b, double* se, double* se_b,
                           void* stream);

/* C in CSR form with r (eqs. 28-30), all outputs device or host, any may be
 * NULL: rowptr [N+1], cols [nnz] (increasing per row), val [nnz], b [N],
 * se [nnz].  Enqueued on `stream`, which is synchronised before returning. */
pdd_status pdd_system_csr(pdd_system sys, int64_t* rowptr, int32_t* cols, double* val, double* b, double* se,
                          void* stream);

typedef struct pdd_system_stats {
  int64_t path_steps;      /* Euler steps over all paths                              */
  int64_t paths;           /* paths simulated                                         */
  int64_t capped_paths;    /* paths stopped by the step cap                           */
  int32_t breakdowns;      /* zero pivots / non-SPD Gram matrices                      */
  int32_t n_launch_spectral, n_launch_mc;
  float ms_sample, ms_build, ms_lu, ms_solve, ms_eval, ms_mc, ms_total;
  int64_t factor_bytes;    /* LU factor bytes kept on the device for the backward pass */
  int32_t recompute;       /* 1: keep_factors asked for more than hbm_budget_bytes, so
                              the backward pass rebuilds the factors chunk by chunk   */
  int32_t n_groups;        /* groups of circles (see the schedule above)              */
  int32_t mixed_buckets;   /* schedule used (chosen by the autotuner for            */
  int32_t grid_cap;        /*   PDD_PLAN_AUTOTUNED)                                    */
  int32_t graph_replays;   /* LU launch sequences replayed from a captured graph     */
  float ms_autotune;       /* time spent tuning in this call (0 when cached)         */
  int64_t gamma_exits;     /* Monte Carlo paths that exited on the interface Gamma_m  */
  int32_t lu_lookahead;    /* 1: the LU launches used the look-ahead stream           */
  int32_t mc_after_floating; /* 1: the Monte Carlo rows ran after the floating rows
                              instead of beside them (PDD_PLAN_AUTOTUNED does so when
                              the previous assembly on the cover found the Monte Carlo
                              work at least 0.8 times as long as the floating rows:
                              the LU launches then only wait for it to free the CUs) */
} pdd_system_stats;

pdd_status pdd_system_get_stats(pdd_system sys, pdd_system_stats* out);

/* ------------------------------------------------------------------ solve */

enum { PDD_SOLVE_BICGSTAB = 0, PDD_SOLVE_DIRECT_SMALL = 1 };

typedef struct pdd_solve_opts {
  double rtol;             /* relative residual |r - C u| / |r|, default 1e-12         */
  int32_t max_iter;        /* default 2000                                             */
  int32_t use_guess;       /* start from the contents of u (BiCGStab)                  */
  int32_t method;          /* PDD_SOLVE_BICGSTAB (default) or PDD_SOLVE_DIRECT_SMALL    */
  int32_t reserved;
} pdd_solve_opts;

typedef struct pdd_solve_info {
  int32_t iterations;
  int32_t converged;
  double rel_residual;
} pdd_solve_info;

/*
 * pdd_solve_G -- solves the assembled system C u = r (eqs. 28-30; Section 4
 * and Remark 2 on solving it) or the transposed system C^T lambda = g of the
 * adjoint (transpose = 1).
 *   rhs  device [N] or NULL for r;  u  device [N] output (and guess).
 *   PDD_SOLVE_BICGSTAB: BiCGStab from u = 0 (or the guess) until
 *     |rhs - C u| <= rtol |rhs|, at most max_iter iterations.  The stream is
 *     synchronised once per 8 iterations (the convergence record of batch k
 *     is read while batch k + 1 runs).
 *   PDD_SOLVE_DIRECT_SMALL: for N <= 4096, [C | rhs] is formed densely on the
 *     device and solved by LU with partial pivoting (the batched LU of the
 *     collocation matrices, one matrix); info->iterations = 1 and
 *     rel_residual = |rhs - C u| / |rhs|.  Allocates about 8 N^2 bytes for
 *     the call; synchronises the stream once.
 * The first BiCGStab solve on a system lays its values out per row (the
 * stencil entries of each row in knot order, the diagonal apart: about
 * 8 nnz bytes, kept with the system) and synchronises the stream; that form
 * serves C and C^T.  Under rule AVERAGED (several stencils per row) C keeps
 * its CSR form and the first transposed solve forms C^T in CSR (pattern per
 * cover, values per system).  Solves on one system may run concurrently on
 * different streams.
 * Errors: PDD_EINVAL (unknown method, N > 4096 for the direct method),
 * PDD_ENOCONV (BiCGStab; u holds the last iterate), PDD_EBREAKDOWN (zero
 * pivot in the direct method), PDD_ENOMEM, PDD_EDEVICE.
 */
pdd_status pdd_solve_G(pdd_system sys, const double* rhs, double* u, int32_t transpose,
                       const pdd_solve_opts* opts, void* stream, pdd_solve_info* info);

/*
 * pdd_solve_G_noalloc -- for callers that cannot allocate device or pinned
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same BiCGStab as pdd_solve_G, with the same kernels
 * and results, but its work area is a fixed 48 MiB array of static device
 * memory, one per GPU, which the library holds until the process ends; the
 * call allocates nothing and creates no events.
 *   Limit: 5 N + 14364 <= 6291456 doubles, i.e. N up to 1255418 knots;
 *   larger systems get PDD_EINVAL.
 *   The operator must already be in its solve form: one pdd_solve_G call on
 *   the system in the same direction builds it (else PDD_EINVAL).
 *   Every call on one GPU uses the same work area and leaves its contents
 *   there; calls that overlap on one GPU (other threads or streams) race and
 *   must be serialised by the caller.
 * Synchronises `stream` once per 8 iterations.
 * Errors: PDD_EINVAL, PDD_ENOCONV (u holds the last iterate), PDD_EDEVICE.
 */
pdd_status pdd_solve_G_noalloc(pdd_system sys, const double* rhs, double* u, int32_t transpose,
                               const pdd_solve_opts* opts, void* stream, pdd_solve_info* info);

/* ------------------------------------------------------- RAS + GMRES */

/*
 * One-level restricted additive Schwarz preconditioner of Section 4
 * (eqs. 42-44):  M^-1 = sum_p R_p^T D_p C_p^-1 R_p,  C_p = R_p C R_p^T.
 * Partition: the circles sorted by centre x (stable) are split into parts_x
 * slabs of near-equal counts (slab s takes sorted positions
 * [s n / parts_x, (s+1) n / parts_x)), each slab sorted by centre y into
 * parts_y parts the same way; empty parts are dropped and the rest numbered
 * in order.  A knot belongs to the part of the circle it lies on; omega_p adds
 * every knot adjacent to one of its knots in the graph of C taken symmetric
 * (one layer).  (D_p)_ii = 1 / (number of omega_q holding knot i), eq. 43.
 * Each C_p (at most 4096 knots) is factorised on the device by LU with partial
 * pivoting and kept as its explicit inverse; HBM use is about 8 (#omega_p)^2
 * bytes per part (4 with fp32_inverses), 16 during the set-up.  The preconditioner refers to `sys`, which must outlive it.
 * With parts_x = parts_y = 1 (N <= 4096) the preconditioner is C^-1 itself and
 * pdd_solve_gmres becomes a direct solve (one iteration).
 * Errors: PDD_EINVAL (bad counts, a part above 4096 knots), PDD_EBREAKDOWN
 * (a singular C_p), PDD_ENOMEM, PDD_EDEVICE.  Synchronises `stream`.
 */
typedef struct pdd_ras_s* pdd_ras;
typedef struct pdd_ras_opts {
  int32_t parts_x, parts_y;   /* >= 1 each                                        */
  int32_t fp32_inverses;      /* 1: keep C_p^-1 rounded to FP32 (half the bytes per
                                 apply; products still accumulate in FP64)        */
  int32_t reserved;
} pdd_ras_opts;

pdd_status pdd_ras_build(pdd_system sys, const pdd_ras_opts* opts, void* stream, pdd_ras* out);

/* Parts (host outputs, any may be NULL): n_parts; omega_off [n_parts+1];
 * omega [omega_off[n_parts]] the sorted knots of each omega_p, concatenated. */
pdd_status pdd_ras_get_parts(pdd_ras ras, int32_t* n_parts, int64_t* omega_off, int32_t* omega);

/* y = M^-1 x (device [N] each, distinct), enqueued on `stream`. */
pdd_status pdd_ras_apply(pdd_ras ras, const double* x, double* y, void* stream);

void pdd_destroy_ras(pdd_ras ras);

typedef struct pdd_gmres_opts {
  double rtol;             /* |g_{j+1}| / |r| (the residual of C u = r), default 1e-12 */
  int32_t max_iter;        /* default 2000                                             */
  int32_t restart;         /* Krylov dimension m, default 30, at most 200              */
} pdd_gmres_opts;

/*
 * pdd_solve_gmres -- restarted GMRES(m) on C u = r with the preconditioner on
 * the right (eq. 45): C M^-1 t = r, u = M^-1 t; ras NULL solves without one.
 * Zero initial guess; Arnoldi by classical Gram-Schmidt applied twice; the
 * Givens rotations and the convergence test run on the device, and `stream`
 * is synchronised once per 8 iterations and once per restart.
 *   rhs  device [N] or NULL for r;  u  device [N] output.
 * Errors: PDD_EINVAL, PDD_ENOCONV (u holds the last iterate), PDD_ENOMEM,
 * PDD_EDEVICE.
 */
pdd_status pdd_solve_gmres(pdd_system sys, pdd_ras ras, const double* rhs, double* u,
                           const pdd_gmres_opts* opts, void* stream, pdd_solve_info* info);

/*
 * pdd_assemble_G_backward -- gradients of a loss L(u) with respect to the
 * node samples of pdd_samples and to r, given u (C u = r) and
 * lambda = C^-T dL/du (device [N] each).  It differentiates the floating
 * rows: the local problems of eqs. 32 and 35 discretised by eq. 40 and
 * solved as in eq. 41, evaluated at the knots (eq. 33).  For floating circle
 * m with mu = A_II^-T E_m^T lambda_Km (E_m the evaluation at its knots):
 *   dL/d coef_q = -mu_q (row q of the operator multiplying coef) . [w_I; w_B]
 *   dL/d f_q    = -mu_q
 * with w_B = H u_Xi and w_I the local interior solution.  Outputs are device
 * arrays [sum_n] in the node layout; NULL skips one.  g_r (device [N], NULL
 * skips it) receives dL/dr = lambda: the Monte Carlo and boundary rows
 * (eqs. 29-30) do not depend on node samples, and their expectations enter
 * only through r.  Needs the system to have been assembled with
 * keep_factors (stored factors, or a chunked recomputation when they
 * exceeded hbm_budget_bytes).  Stream-ordered; synchronises the stream only
 * to release chunk buffers (recomputation, rule AVERAGED).
 * Errors: PDD_EINVAL (no factors kept, a bucket whose adjoint layout exceeds
 * the 160 KiB of LDS), PDD_ENOMEM, PDD_EDEVICE.
 */
pdd_status pdd_assemble_G_backward(pdd_system sys, const double* u, const double* lambda,
                                   double* g_axx, double* g_axy, double* g_ayy,
                                   double* g_bx, double* g_by, double* g_c, double* g_f,
                                   double* g_r, void* stream);

void pdd_destroy_system(pdd_system sys);

#ifdef __cplusplus
}
#endif

#endif /* PDD_H */
