/*
 * mlmc.h -- C ABI of the MI355X (gfx950) multilevel Monte Carlo sample-solve library.
 *
 * The library runs the per-sample work of the multilevel Monte Carlo method of
 * Dodwell, Kynaston, Butler, Haftka, Kim and Scheichl, "Multilevel Monte Carlo
 * Simulations of Composite Structures with Uncertain Manufacturing Defects":
 *
 *   - KL synthesis of a random fibre-angle field (Section 3.1, Eq. inftyKL);
 *   - finite-element solves of an orthotropic strip with that field
 *     (Section 3.1, Eq. matrixinplane) and its quantity of interest, for a
 *     plane-stress strip (u, v per node) or the paper's Cosserat continuum
 *     (u, v, theta_3 per node, strength from Eq. failureCriterion);
 *   - smallest buckling load of a laminated plate with random ply angles
 *     (Section 4.1, Eqs. CLTABD, MomentWeakForm, matrixeig);
 *   - FP64 level sums for the estimators of Section 2 (Eqs. MLMC_defn,
 *     varianceestim, biased_estimator).
 *
 * A sample Y_l = Q_l - Q_{l-1} needs two solves on consecutive levels with the
 * same random parameters (Section 2.2, after Eq. MLMC_defn); a "coupled"
 * request does both in one call.
 *
 * Conventions shared by every entry point
 *   - Status: functions return MLMC_OK (0) or a negative mlmc_status.  The text
 *     of the last error of a context is returned by mlmc_last_error().  Argument
 *     errors are detected before any device work is queued.
 *   - Numerical failures of single samples (no convergence, NaN, breakdown) do
 *     not fail a call; they are reported per sample in mlmc_info.status_*.
 *   - Pointers marked "dev" are device (HBM) addresses of the current HIP
 *     device; "host" pointers are ordinary host memory.  The caller owns every
 *     buffer it passes; the context owns its tables and workspaces.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *     is queued on it; functions returning device results are asynchronous
 *     unless stated otherwise.
 *   - One context must not be used from two host threads at once.
 *   - Results of a sample depend only on (configuration, level, its parameter
 *     row, precision, rtol): not on the other samples of the batch.
 */
#ifndef MLMC_H
#define MLMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlmc_ctx mlmc_ctx;

typedef enum {
  MLMC_OK = 0,
  MLMC_EINVAL = -1, /* bad argument or configuration */
  MLMC_ENOMEM = -2, /* request exceeds the memory budget or device memory */
  MLMC_EHIP = -3,   /* a HIP runtime call failed */
  MLMC_ESTATE = -4  /* call not valid for this context (e.g. plate call on a strip config) */
} mlmc_status;

typedef enum { MLMC_FP64 = 0, MLMC_MIXED = 1 } mlmc_precision;

typedef enum {
  MLMC_S_OK = 0,        /* converged */
  MLMC_S_NOCONV = 1,    /* iteration limit reached */
  MLMC_S_NAN = 2,       /* NaN/Inf met (e.g. non-finite parameters) */
  MLMC_S_BREAKDOWN = 3, /* p^T A p <= 0 or a singular Rayleigh-Ritz step */
  MLMC_S_SKIPPED = 4,   /* not solved (coarse part of a level-0 request) */
  MLMC_S_NOTLOWEST = 5  /* buckling: converged, but a lower eigenvalue exists (the
                           lowest-mode check of mlmc_buckle_batch failed) */
} mlmc_sample_status;

/* One sample request: row `sample` of the parameter array, mesh level `level`;
 * `coupled` != 0 also solves level-1 with the same row (a Y_l sample). */
typedef struct {
  int64_t sample;
  int32_t level;
  int32_t coupled;
} mlmc_request;

/* Per-request solver report (32 bytes, no implicit padding). */
typedef struct {
  int32_t iters_f, iters_c;   /* iterations of the fine / coarse solve      */
  double relres_f, relres_c;  /* final recursive ||r||/||b|| (or eigen res) */
  int32_t status_f, status_c; /* mlmc_sample_status of each solve           */
} mlmc_info;

/* FP64 accumulator of one level (Section 2.3: N_l, sums of Y and Y^2 for the
 * sample mean and Eq. varianceestim; failure counts for Eq. biased_estimator).
 * Sums are Neumaier-compensated: the value is sum + comp. */
typedef struct {
  int64_t n, n_plus, n_minus;
  double sum_y, sum_y2, sum_qf, sum_qc, sum_cost;
  double comp_y, comp_y2, comp_qf, comp_qc;
} mlmc_level_acc;

/* ---------------------------------------------------------------- lifecycle */

/* Create a context on the current HIP device from a JSON workload definition
 * ("kind": "strip", "cosserat" or "plate"; mesh hierarchy, material,
 * covariance, solver settings).  Builds the level hierarchy (Section 2.3: uniform refinement),
 * the KL mode tables of every level (Section 3.1) and, for plates, the
 * laminate data (Section 4.1).  `mem_budget_bytes` bounds the workspaces the
 * context may allocate later (0 = 90% of free device memory).
 * Errors: MLMC_EINVAL (bad JSON / values), MLMC_EHIP, MLMC_ENOMEM.
 * On error *out is NULL; the message is available from mlmc_last_error(NULL). */
int mlmc_create(const char *config_json, size_t mem_budget_bytes, mlmc_ctx **out);

/* Free every device buffer of the context.  NULL is ignored. */
void mlmc_destroy(mlmc_ctx *ctx);

/* Last error text of `ctx` (or of the last failed mlmc_create if ctx == NULL).
 * The string stays valid until the next call on the same context. */
const char *mlmc_last_error(const mlmc_ctx *ctx);

/* Number of levels and per-level sizes of the context's hierarchy:
 * nodes, dofs (unknowns incl. constrained ones), elements, Gauss points. */
int mlmc_level_info(const mlmc_ctx *ctx, int level, int64_t *n_nodes, int64_t *n_dofs,
                    int64_t *n_elem, int64_t *n_gp);
int mlmc_num_levels(const mlmc_ctx *ctx);

/* Device bytes one in-flight request of `kind` (0 strip, 1 plate) at `level`
 * needs in the given precision (workspace slots, excluding caller buffers).
 * Used for admission by memory footprint. */
int mlmc_footprint(const mlmc_ctx *ctx, int kind, int level, int precision, size_t *bytes_per_request);

/* Allocate the workspace for `n` requests of `level` in `precision` now, so that
 * later batches of up to `n` requests of that level allocate nothing (a level's
 * workspace serves both the fine solves of its requests and the coarse solves
 * of coupled requests one level up).  The workspace only grows; the total of
 * all levels stays within the context's budget.
 * Errors: MLMC_EINVAL (level, n < 0, precision), MLMC_ENOMEM (budget or
 * device memory), MLMC_EHIP. */
int mlmc_reserve(mlmc_ctx *ctx, int level, int n, int precision);

/* ----------------------------------------------------------- strip (Test I) */
/* The strip calls below serve two models.  A "strip" context solves the
 * plane-stress orthotropic strip: unknowns (u, v) per node.  A "cosserat"
 * context solves the Cosserat continuum of Section 3.1 (Eqs. VarCosserat,
 * matrixinplane): unknowns (u, v, theta_3) per node (n_dofs = 3 n_nodes), the
 * fibre-frame matrices C (4 x 4 on the non-symmetric strains eps_11, eps_22,
 * eps_12, eps_21) and D (2 x 2 on the curvatures) rotated by the angle field,
 * u = 0 on x = 0, u = delta on x = L, v = 0 on y = 0 and y = L; its level l
 * uses the first 50 + 50 l (configurable) KL terms of the parameter row; its
 * quantity of interest is the compressive strength of Eq. failureCriterion;
 * it is solved in FP64 only (MLMC_MIXED gives MLMC_EINVAL) and its fields
 * are written in FP64 only. */

/* KL synthesis (Eq. inftyKL truncated after the configured number of modes,
 * plus the optional wrinkle A sech^2((x - x0)/w)) at the 2x2 Gauss points of
 * `level`.  xi: dev [n][ld_xi] FP64 rows [xi_1..xi_K, A, x0, w] (K = modes).
 * theta: dev [n][n_gp(level)], element-major, Gauss points in the order
 * (-,-), (+,-), (-,+), (+,+); dtype 0 = FP64, 1 = BF16 (round to nearest even).
 * Angles in radians.  Errors: MLMC_EINVAL (level, n < 0, ld_xi < K + 3). */
int mlmc_sample_field(mlmc_ctx *ctx, int level, int n, const double *xi, int ld_xi, void *theta,
                      int dtype, void *stream);

/* Matrix-free operator of the strip at `level` (Section 3.1: bilinear elements,
 * 2x2 Gauss, rotated ply stiffness at each Gauss point):
 *   y = P K(theta) P x + (I - P) x,
 * P = projector on the unconstrained unknowns (left edge u = v = 0, right edge
 * u prescribed).  `raw` != 0 applies K(theta) without the projection.
 * theta: dev [n][n_gp] FP64; x, y: dev [n][n_dofs] FP64, unknowns interleaved
 * (u, v) per node, node (i, j) at index j (nx + 1) + i. */
int mlmc_strip_apply(mlmc_ctx *ctx, int level, int n, const double *theta, const double *x, double *y,
                     int raw, void *stream);

/* Dirichlet lifting and Jacobi diagonal: b = -P K g (g = prescribed values:
 * u = -delta on the right edge) and dinv = 1 / diag(P K P + I - P).
 * theta: dev [n][n_gp]; b, dinv: dev [n][n_dofs]. */
int mlmc_strip_rhs_diag(mlmc_ctx *ctx, int level, int n, const double *theta, double *b, double *dinv,
                        void *stream);

/* Solve K(theta) d = f for each of n given fields (Jacobi-PCG, x0 = 0, stop at
 * ||r||_2 <= rtol ||b||_2 on the recursive residual) and evaluate the quantity
 * of interest: max over the Gauss points of the elements with centroid in the
 * configured central region of the compressive stress along the local fibre
 * direction.  theta: dev [n][n_gp] FP64; q: dev [n]; info: dev [n] (fine fields
 * of mlmc_info are filled); d (optional, may be NULL): dev [n][n_dofs] total
 * displacement.  precision: MLMC_FP64 or MLMC_MIXED.  Synchronous. */
int mlmc_strip_solve_theta(mlmc_ctx *ctx, int level, int n, const double *theta, double *q, double *d,
                           mlmc_info *info, int precision, double rtol, void *stream);

/* Size of the fixed per-GPU scratch array of mlmc_strip_solve_theta_noalloc. */
#define MLMC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * form of mlmc_strip_solve_theta, with every workspace buffer of the solve
 * carved from one fixed device array of MLMC_SCRATCH_BYTES per GPU (part of
 * the library's code object, held until the process ends) instead of the
 * context's pool.  The call allocates nothing: no hipMalloc, hipFree, pinned
 * host memory, events or graphs (event timing and graph replay are off for
 * the call).
 * theta: dev [n][n_gp] FP64 angles; q: dev [n] quantities of interest; info:
 * dev [n] (fine fields filled; may be NULL); rtol <= 0 uses the configured
 * tolerance.  Results are bit-identical to mlmc_strip_solve_theta in FP64.
 * The context's device must be current.  Every call on a GPU shares that
 * GPU's array, whatever the context: calls that overlap on one GPU (two host
 * threads, or two streams without ordering between the calls) race and give
 * wrong results.  The call clears the part of the array it uses before the
 * solve and synchronises `stream` before returning.
 * Errors: MLMC_EINVAL (level, n < 0, null pointers), MLMC_ESTATE (plate
 * context, another device current), MLMC_ENOMEM (n solves of `level` need more
 * than MLMC_SCRATCH_BYTES, or n > 4096; nothing is queued then), MLMC_EHIP. */
int mlmc_strip_solve_theta_noalloc(mlmc_ctx *ctx, int level, int n, const double *theta, double *q,
                                   mlmc_info *info, double rtol, void *stream);

/* Sample solves: for request i, Q at req[i].level from parameter row
 * xi[req[i].sample] (and Q at level - 1 with the same row when coupled and
 * level > 0).  req: host [n_req]; xi: dev [n_rows][ld_xi] (every req[i].sample
 * must be in [0, n_rows), else MLMC_EINVAL); q_fine, q_coarse:
 * dev [n_req] (q_coarse[i] = 0 and status_c = MLMC_S_SKIPPED when not
 * coupled or level 0); info: dev [n_req].  rtol <= 0 uses the configured
 * tolerance.  Synchronous with respect to `stream` on return. */
int mlmc_solve_batch(mlmc_ctx *ctx, int n_req, const mlmc_request *req, const double *xi, int64_t n_rows,
                     int ld_xi, double *q_fine, double *q_coarse, mlmc_info *info, int precision, double rtol,
                     void *stream);

/* ---------------------------------------------------------- plate (Test II) */

/* Smallest positive lambda of K phi = lambda K_G phi (Eq. matrixeig) for the
 * laminate of each request: pristine ply angles plus the row
 * ply_offsets[req[i].sample] (radians, dev [n_rows][n_plies], rows checked as
 * for mlmc_solve_batch); coupled requests
 * also solve level - 1.  lam_fine, lam_coarse: dev [n_req] in N/mm of edge
 * load; tol: relative eigen-residual (<= 0: configured).  Synchronous.
 * Lowest-mode check (on unless the workload sets "cert_shift": 0): after a
 * solve converges, the band of K - sigma K_G with sigma = lambda (1 -
 * cert_shift) (default 1e-6) is factored in FP64; since K is positive
 * definite and K_G semi-definite on the free unknowns, a factorisation without
 * a non-positive pivot shows that no eigenvalue lies below lambda (1 -
 * cert_shift).  A sample that fails the check keeps its lambda and gets
 * status MLMC_S_NOTLOWEST.  "eig_start_p0" (default 0: the integer nearest to
 * a / b) sets the half-waves along x of the first start vector. */
int mlmc_buckle_batch(mlmc_ctx *ctx, int n_req, const mlmc_request *req, const double *ply_offsets,
                      int64_t n_rows, double *lam_fine, double *lam_coarse, mlmc_info *info, int precision,
                      double tol, void *stream);

/* Matrix-free plate operators for one sample per row of ply_offsets (dev
 * [n][n_plies], radians): y = P K P x (geometric == 0) or y = P K_G P x
 * (geometric != 0), with P the projector on the unconstrained unknowns
 * (Section 4.1: Reissner-Mindlin Q4, selective reduced integration, or the
 * MITC4 assumed transverse shear strain when the workload sets
 * "shear": "mitc4"; laminate [[A, B], [B, D]], or [[A, 0], [0, D*]] with
 * D* = D - B^T A^-1 B when it sets "condensed": true; K_G = int N0 w_x w_x).  x, y: dev [n][5 n_nodes], unknowns (u, v, w,
 * theta_x, theta_y) per node, node (i, j) at j (nx + 1) + i; y = 0 on
 * constrained unknowns. */
int mlmc_plate_apply(mlmc_ctx *ctx, int level, int n, const double *ply_offsets, int geometric, const double *x,
                     double *y, void *stream);

/* ------------------------------------------------------------- level sums */

/* Accumulate one batch of a level into `acc` (host, in/out), in FP64 with a
 * fixed summation order: Y = q_fine - q_coarse (q_coarse may be NULL: Y =
 * q_fine, as for level 0 where Y_0 = Q_0).  If lambda_star is not NaN the
 * inputs are buckling loads and are first turned into failure indicators
 * 1(lambda < lambda_star) (Section 2.4); n_plus / n_minus count Y = +1 / -1.
 * cost_per_sample is added n times to sum_cost.  q_fine, q_coarse: dev [n].
 * Synchronises `stream` before returning. */
int mlmc_level_stats(mlmc_ctx *ctx, int level, int n, const double *q_fine, const double *q_coarse,
                     double cost_per_sample, double lambda_star, mlmc_level_acc *acc, void *stream);

/* ------------------------------------------------------------ diagnostics */

/* Kernel timing for roofline measurement.  While enabled, the launches of the
 * two PCG passes (kernel 0: operator pass, fused p-update + A p + p.Ap;
 * kernel 1: vector pass, x/z update + r.z, r.r) of one iteration in the
 * middle of every block of 32 iterations are bracketed by HIP events on the
 * stream of the solve (timing every launch would slow the solve by about 7%):
 * iteration 16 of even blocks and 17 of odd ones, so that both forms of the
 * vector pass are sampled.
 * mlmc_profile_read returns the summed event time (ms) and the number of
 * those timed launches, and the algorithmic HBM bytes of exactly those
 * launches (the bytes each sample active in the timed iteration must move;
 * the residual is kept preconditioned, z = r / diag(A):
 * operator pass reads z, p and writes A p, 3 vectors of 16 B/node, plus
 * 32 B/element of angle codes or 64 B/element of pairs; vector pass reads x,
 * z, p, A p, diag(A) and writes x, z, p, 8 vectors of 16 B/node, x only at
 * odd iterations).  Results are unchanged. */
int mlmc_profile_enable(mlmc_ctx *ctx, int on);
/* kernel: 0 / 1 = FP64 operator / vector pass, 2 / 3 = the FP32 passes of the
 * mixed-precision inner solver (3 vectors of 8 B/node + 16 B/element of FP32
 * angles, or 8 B/element with "theta_storage": "bf16", and 8 vectors of
 * 8 B/node).  kernel + 4 (4..7): the same launches, with *alg_bytes set to
 * the number of unknowns (dofs) the active samples of those launches hold,
 * the unit of per-unknown byte figures. */
int mlmc_profile_read(mlmc_ctx *ctx, int kernel, double *total_ms, int64_t *launches, double *alg_bytes);

#ifdef __cplusplus
}
#endif

#endif /* MLMC_H */
