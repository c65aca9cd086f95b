/*
 * igamg — multigrid solver for multi-patch isogeometric discretizations of the
 * Poisson problem on AMD Instinct MI355X (gfx950).
 *
 * Method: S. Takacs, "Fast multigrid solvers for conforming and non-conforming
 * multi-patch Isogeometric Analysis" (arXiv:1902.01818).
 *   - model problem -Delta u = f, u = 0 on the boundary: Section 2, eq. model
 *   - patches G_k:(0,1)^d -> Omega_k, tensor B-splines of degree p, maximum
 *     smoothness: Section 2, eqs. omega:1, omega:2, local
 *   - conforming space: Section 2, eq. igaspace0; SIPG space and bilinear
 *     form: Section 3, eqs. igaspace, model:discr2, penalty of the finest grid
 *     on every level: eq. a:galerkin
 *   - V-cycle: Algorithm 1; hybrid smoother: Algorithm 2 (Section 6);
 *     Gauss-Seidel: Section 4; subspace corrected mass smoother: Section 5,
 *     eq. Ldef; stopping rule and PCG: Section 4.
 *
 * Conventions common to all entry points
 *   - Every function returns an int status: 0 = success, < 0 = error,
 *     > 0 = warning (IGAMG_ENOCONV).  No C++ exception crosses this boundary.
 *     igamg_last_error() returns a thread-local message for the last error.
 *   - Vectors passed to the device entry points are caller-owned device
 *     pointers (float64, contiguous), in the compact ordering: patches in array
 *     order, inside a patch lexicographic with x fastest, unknowns with a
 *     non-zero trace on the boundary skipped; in the conforming case a glued
 *     interface unknown keeps the index of its first visit.  Several
 *     right-hand sides are stored one after the other ([nrhs][N]).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Device entry
 *     points are asynchronous on that stream unless stated otherwise.
 *   - A context owns all device memory it allocates; igamg_destroy frees it.
 *     A context must not be used from two host threads at the same time.
 */
#ifndef IGAMG_H
#define IGAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define IGAMG_OK 0
#define IGAMG_EINVAL (-1)       /* invalid argument or geometry */
#define IGAMG_EUNSUPPORTED (-2) /* valid input this library does not handle */
#define IGAMG_ENOMEM (-3)       /* device allocation failed / over budget */
#define IGAMG_EHIP (-4)         /* HIP runtime error */
#define IGAMG_ENOCONV 1         /* warning: tolerance not reached in maxit */

/* discretization (Sections 2 and 3) */
#define IGAMG_SIPG 0
#define IGAMG_CONFORMING 1
/* smoother: Algorithm 2 (hybrid), Algorithm 1 with eq. Ldef (SCMS), Section 4 (GS) */
#define IGAMG_SMOOTHER_HYBRID 0
#define IGAMG_SMOOTHER_SCMS 1
#define IGAMG_SMOOTHER_GS 2
/* Arithmetic of the cycle.  The outer iteration, its residuals, the
 * convergence test and the coarsest-level solve are float64 always; with
 * IGAMG_FP32 every other kernel of the cycle stores and computes in float32
 * (operator data rounded once at setup), i.e. the cycle is a float32
 * preconditioner inside a float64 Krylov iteration (an extension beyond the
 * paper, which computes in float64 throughout). */
#define IGAMG_FP64 0
#define IGAMG_FP32 1
/* float32 cycle as IGAMG_FP32 whose patch-interior solves of the subspace
 * corrected mass smoother (Section 5, eq. Ldef, fast diagonalization) round
 * their contraction operands to bfloat16 (nearest even) and accumulate in
 * float32 on the matrix cores.  The eigenvector matrices are rounded once,
 * the same rounded matrix serving both directions, so the interior solve
 * stays symmetric in exact arithmetic; the outer iteration should be
 * IGAMG_OUTER_FCG. */
#define IGAMG_BF16_SCMS 2
/* Outer iteration: PCG preconditioned by one cycle (Section 4); the cycle
 * used directly as the solver (Section 4); flexible CG (Polak-Ribiere beta,
 * robust to a preconditioner that is not exactly symmetric, e.g. float32). */
#define IGAMG_OUTER_PCG 0
#define IGAMG_OUTER_MG 1
#define IGAMG_OUTER_FCG 2
/* Iterative refinement: x <- x + d with d an inner PCG solve of A d = f - A x
 * (the residual in float64) whose operator applies and preconditioning cycle
 * run in the cycle arithmetic, stopped at a 1e-4 relative reduction of the
 * inner residual; the outer loop stops on the float64 residual.  maxit bounds
 * the total inner iterations of each right-hand side; `iterations` reports
 * that total (one cycle each). */
#define IGAMG_OUTER_IR 3
/* Operator applies (the cycle's residuals and the float64 outer apply).
 * AUTO: from the stored matrix rows on the levels that keep them (SIPG with
 * a Gauss-Seidel smoother keeps the rows of every level above the coarsest:
 * (2p+1)^2 same-patch entries per unknown plus the cross-patch couplings),
 * by sum factorization elsewhere.  SUMFACT: matrix-free everywhere (eq.
 * model, Section 2, evaluated by sum factorization; the SIPG interface terms
 * of Section 3 as a sparse gather).  ROWS: the stored rows wherever the
 * cycle has them; setup fails with IGAMG_EUNSUPPORTED when it has none.  In
 * float32 cycles the rows also keep a float64 copy on the finest level for
 * the outer apply.  Both forms apply the same matrix (assembled with the
 * same quadrature); their results differ by rounding only. */
#define IGAMG_APPLY_AUTO 0
#define IGAMG_APPLY_SUMFACT 1
#define IGAMG_APPLY_ROWS 2

/* Multi-patch geometry (Section 2, eqs. omega:1/omega:2, Assumption 1).
 * Each patch map is the multilinear interpolation of its 2^dim corners; corner
 * b has parameter coordinates (bit_0(b), ..., bit_{dim-1}(b)), x fastest.
 * Patches that share a full side must traverse it with the same orientation.
 * All pointers are host pointers, read during igamg_setup only. */
typedef struct {
  int dim;                /* 2 or 3 */
  int n_patches;          /* K >= 1 */
  const double *corners;  /* [n_patches][2^dim][dim] */
  const int32_t *elems;   /* [n_patches][dim] elements per direction on the finest level */
  const int32_t *degrees; /* [n_patches] spline degree per patch, or NULL: `degree` of
                             igamg_setup on every patch.  Different degrees (the
                             non-matching spaces of Section 5) take the SIPG space with
                             the SCMS smoother in 2D; the penalty of an interface uses
                             the larger degree of its two sides */
} igamg_patches;

typedef struct {
  int discretization; /* IGAMG_SIPG or IGAMG_CONFORMING */
  int smoother;       /* IGAMG_SMOOTHER_* */
  int mu;             /* 1 = V-cycle, 2 = W-cycle (Algorithm 1) */
  int nu;             /* smoothing steps (Algorithm 1/2) */
  double damping_tau; /* tau of eq. Ldef */
  double scaling_delta; /* SCMS scaling sigma = 1/(delta h^2), Section 5 */
  int precision;      /* IGAMG_FP64 / IGAMG_FP32 / IGAMG_BF16_SCMS (cycle arithmetic) */
  int outer;          /* IGAMG_OUTER_* */
  int gs_tile;        /* Gauss-Seidel tile width T >= p of the colour ordering, 0 = 2(p+1) */
  int coarse_min;     /* halve element counts while all are even and their half >= coarse_min; 0 = 2 */
  int timing;         /* 1 = record per-kernel-family event timings (igamg_kernel_stats) */
  int max_rhs;        /* right-hand sides processed together by one call (work-vector
                         capacity, 0 = 1); larger nrhs are split into batches of max_rhs */
  int operator_apply; /* IGAMG_APPLY_* */
  int graphs;         /* 1 = replay the outer iteration's preconditioner cycle (one per
                         residual vector and batch size) from a HIP graph captured at
                         its second use (the first runs launch by launch); 0 = launch
                         kernel by kernel.  Ignored while timing is on */
} igamg_options;

typedef struct {
  int iterations;          /* outer iterations performed */
  double rel_residual;     /* ||r_k|| / ||f|| of the outer recurrence at exit */
  double true_rel_residual;/* ||f - A u|| / ||f|| recomputed in float64 at exit */
  double seconds;          /* wall time of the solve on the host */
  double *history;         /* optional host array [maxit+1] of relative residuals, or NULL
                              (entry k after outer iteration k; with IGAMG_OUTER_IR after
                              refinement step k, the float64 residual) */
} igamg_solve_info;

typedef struct igamg_ctx igamg_ctx;

/* Fill *o with the defaults (SIPG, hybrid, V(1,1), tau 0.25, delta 0.1, FP64, PCG,
 * one right-hand side per batch, operator applies IGAMG_APPLY_AUTO, no graphs). */
void igamg_default_options(igamg_options *o);

/* Host only, no GPU work: device bytes igamg_setup will allocate for this
 * problem with a batch capacity of nrhs right-hand sides (nrhs >= 1; 0 =
 * o->max_rhs), used for admission by memory footprint.  An estimate from the
 * sizes of every array setup allocates, with a 15 % margin.
 * Errors: IGAMG_EINVAL. */
int igamg_footprint(const igamg_patches *patches, int degree, const igamg_options *o, int nrhs,
                    size_t *bytes);

/* Build the grid hierarchy (uniform dyadic refinement, Section 2), the
 * operators of every level (SIPG: penalty sigma p^2/h with the finest h,
 * eq. a:galerkin), transfer operators (canonical embedding, Section 4),
 * smoother data (Section 5: SCMS factors, dense inverses of the interface
 * pieces P^T A P; Section 4: Gauss-Seidel colouring and stencil rows) and
 * the dense inverse of the coarsest matrix (blocked Gauss-Jordan in
 * float64; the paper fixes only a direct solve there).
 * degree >= 1; penalty_sigma > 0 (SIPG only).  Synchronizes `stream`.
 * dim 3 takes degree 1..4 (higher degrees return IGAMG_EUNSUPPORTED).
 * Errors: IGAMG_EINVAL (dim, degree, non-positive Jacobian, conforming
 * interface mismatch), IGAMG_EUNSUPPORTED (flipped interface orientation,
 * Gauss-Seidel with the conforming space, 3D degree above 4),
 * IGAMG_ENOMEM, IGAMG_EHIP.
 * On success *out owns the context. */
int igamg_setup(const igamg_patches *patches, int degree, double penalty_sigma,
                const igamg_options *o, void *stream, igamg_ctx **out);

/* Number N of unknowns on the finest level (compact ordering). */
int igamg_num_dofs(const igamg_ctx *ctx, int64_t *n);
/* Number of grid levels L+1. */
int igamg_num_levels(const igamg_ctx *ctx, int *levels);

/* y = A_L x (eq. linear:system / linear:system:0), float64; x, y device [nrhs][N].
 * With IGAMG_APPLY_AUTO the finest level's stored rows are applied where the
 * level keeps them (SIPG with a Gauss-Seidel smoother), otherwise the volume
 * part is evaluated matrix-free by sum factorization (see IGAMG_APPLY_*). */
int igamg_apply(igamg_ctx *ctx, const double *x, double *y, int nrhs, void *stream);

/* One multigrid cycle u <- MG(L, f, u) (Algorithm 1 or 2 per options), u
 * in/out, f in; device [nrhs][N]; internal arithmetic per o->precision.
 * Right-hand sides go through the cycle max_rhs at a time (one launch per
 * kernel and batch). */
int igamg_vcycle(igamg_ctx *ctx, const double *f, double *u, int nrhs, void *stream);

/* Solve A_L u = rhs until ||rhs - A u|| / ||rhs|| <= tol (Section 4) with the
 * outer iteration of the options (PCG or flexible CG preconditioned by one
 * cycle, or the cycle used directly); the residual tested is the float64
 * recurrence residual of the outer iteration.  u: device in/out (initial
 * guess used if use_initial_guess, else zero).  info: host array [nrhs] or
 * NULL (iterations = the iteration at which that right-hand side met tol).
 * Right-hand sides are solved max_rhs at a time, each with its own scalars;
 * a converged one is frozen while the rest of its batch iterates.
 * Synchronizes `stream` once per outer iteration (convergence test).
 * Returns IGAMG_ENOCONV if a right-hand side missed tol within maxit; u then
 * holds its last iterate. */
int igamg_solve(igamg_ctx *ctx, const double *rhs, double *u, int nrhs, double tol,
                int maxit, int use_initial_guess, igamg_solve_info *info, void *stream);

/* Manufactured solutions (Section 2, the experiments' choice):
 * IGAMG_MANUFACTURED_SINE: u = prod_d sin(pi x_d), f = -Delta u = d pi^2 u. */
#define IGAMG_MANUFACTURED_SINE 0

/* f_i = (f, phi_i) for the manufactured solution `which`, Gauss quadrature
 * with p+1 points; f device [N].  Errors: IGAMG_EINVAL (null argument,
 * unknown `which`). */
int igamg_load_manufactured(igamg_ctx *ctx, int which, double *f, void *stream);

/* Discretization error ||u_h - u||_{L2(Omega)} of the finest-level
 * coefficient vector u_h (device [N], compact ordering, caller-owned) against
 * the manufactured solution `which` (Section 2, model problem), Gauss
 * quadrature with p+3 points per element and direction, summed in a fixed
 * order.  Writes *err_host (host); synchronizes `stream`; allocates and frees
 * its own scratch.  Errors: IGAMG_EINVAL (null argument, unknown `which`),
 * IGAMG_EHIP. */
int igamg_l2_error(igamg_ctx *ctx, const double *u, int which, double *err_host, void *stream);

/* igamg_l2_error without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and result as
 * igamg_l2_error (the same fixed summation order, so the same value bit for
 * bit).  Its scratch (tables, block partial sums, the result) lives in one
 * static device array of 16 MiB per GPU, held until the process ends; the
 * array's address is looked up once per device by igamg_setup.  Every call
 * on a GPU shares that GPU's array: calls that overlap on one GPU (two
 * streams, two host threads) race and must be serialized by the caller.
 * The current device must be the context's device.  Synchronizes `stream`.
 * Errors: IGAMG_EINVAL (null argument, context of another device),
 * IGAMG_EUNSUPPORTED (the problem's tables and partial sums need more than
 * 16 MiB: about 500 million elements, or very large element counts per patch
 * at high degree), IGAMG_EHIP. */
int igamg_l2_error_noalloc(igamg_ctx *ctx, const double *u, int which, double *err_host,
                           void *stream);

/* Device bytes owned by the context. */
int igamg_memory(const igamg_ctx *ctx, size_t *bytes);

/* Per-kernel-family event timings recorded since the last reset when the
 * context was set up with o->timing = 1.  names: host array of `cap` char
 * buffers of 32 bytes; ms / launches: host arrays [cap].  *count = families
 * written.  reset != 0 clears the counters after reading.  Synchronizes. */
int igamg_kernel_stats(igamg_ctx *ctx, int cap, char (*names)[32], double *ms,
                       int64_t *launches, int *count, int reset);

/* Per-kernel-family event timing filter: families are keyed "<family>/<level>"
 * (e.g. "vol_apply/5"); only keys starting with `filter` are timed ("" = all),
 * filter == NULL switches timing off.  Events are recorded on the launch
 * stream around every matching launch. */
int igamg_set_timing(igamg_ctx *ctx, const char *filter);

/* Algorithmic bytes moved and flops of one timed launch of a kernel family
 * on a level (level < 0: finest) for a batch of nrhs right-hand sides: the
 * roofline model of the library's kernels.  Families: "stencil_apply" and
 * "vol_apply" + "iface_apply" (operator, eq. model:discr2), "outer_apply"
 * (the float64 finest-level operator of a float32-cycle solve),
 * "gauss_seidel" (one colour class), "scms" (one application to all patch
 * interiors, eq. Ldef), "pieces" (all interface pieces), "restrict" /
 * "prolong" (level = the fine side), "coarse" (the direct solve; level
 * ignored).  Operator data shared by the batch counts once; vectors once per
 * right-hand side.  The stored-row operator and Gauss-Seidel count the
 * (2p+1)^d stencil of every compact unknown and three vector accesses per
 * unknown and right-hand side, nothing for padding, masks or index lists.  Errors: IGAMG_EINVAL for an unknown family, a level out
 * of range or nrhs < 1. */
int igamg_kernel_model(igamg_ctx *ctx, const char *family, int level, int nrhs, double *bytes,
                       double *flops);

int igamg_destroy(igamg_ctx *ctx);

/* Host only: number of unknowns N of the finest level (compact ordering) and
 * number of levels of a problem, as igamg_setup would build it.  Errors as
 * igamg_setup's argument checks. */
int igamg_problem_size(const igamg_patches *patches, int degree, const igamg_options *o,
                       int64_t *n_dofs, int *levels);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of independent solve requests on one GPU.
 *
 * A server owns `slots` worker threads, each with its own HIP stream, and
 * one device buffer of `memory_budget` bytes.  Requests are admitted in
 * arrival order as soon as a slot is free and a contiguous block of the
 * buffer holds the request's footprint (igamg_footprint of its problem plus
 * its right-hand side and solution); the request then builds its hierarchy
 * inside that block (setup, as igamg_setup), solves (as igamg_solve with one
 * right-hand side, its preconditioner cycle replayed from a captured HIP
 * graph: option graphs = 1), copies the solution to the host and returns the
 * block.
 * Requests of different patch layouts, degrees and sizes therefore run
 * concurrently on the device, and requests arriving while others run start
 * as slots and memory free up.  The method per request is the one of
 * igamg_solve (Sections 2-6); each result is independent of the other
 * requests in flight (the tests compare a mix with requests run alone).
 * ------------------------------------------------------------------------- */
typedef struct igamg_server igamg_server;

typedef struct {
  int slots;            /* requests on the GPU at the same time (1..64) */
  size_t memory_budget; /* device bytes shared by admitted requests (>= 1 MiB) */
  int device;           /* HIP device ordinal */
} igamg_server_config;

typedef struct {
  int status;              /* status of the request (igamg_solve's, or an error) */
  int iterations;          /* outer iterations */
  double rel_residual;     /* recurrence residual at exit */
  double true_rel_residual;/* float64 ||f - A u|| / ||f|| at exit */
  int64_t n_dofs;          /* N */
  size_t footprint;        /* bytes reserved for the request */
  int fallback_allocations;/* arrays that did not fit the block (allocated by the driver) */
  double t_submit, t_admit, t_ready, t_done; /* seconds since server creation:
                              submitted, admitted, set up (rhs on the GPU), solved */
} igamg_request_info;

/* Create a server (allocates the budget, starts the workers).  Errors:
 * IGAMG_EINVAL, IGAMG_ENOMEM (budget not allocatable), IGAMG_EHIP. */
int igamg_server_create(const igamg_server_config *cfg, igamg_server **out);

/* Queue one request: problem as for igamg_setup (host arrays, copied),
 * options (max_rhs, timing and graphs are ignored; precision must be IGAMG_FP64,
 * float32 requests return IGAMG_EUNSUPPORTED), rhs = host float64 array of
 * n_dofs values (copied; n_dofs must equal igamg_problem_size's N), tol and
 * maxit as for igamg_solve.  Returns at once with *request_id.  Input errors
 * are returned here; setup/solve errors are reported by igamg_server_wait. */
int igamg_server_submit(igamg_server *srv, const igamg_patches *patches, int degree,
                        double penalty_sigma, const igamg_options *o, const double *rhs,
                        int64_t n_dofs, double tol, int maxit, int64_t *request_id);

/* Block until the request is done; copy its solution to host array u (n_dofs
 * values, may be NULL) and its record to *info (may be NULL); release the
 * request.  Returns the request's status (IGAMG_ENOMEM if its footprint
 * exceeds the whole budget). */
int igamg_server_wait(igamg_server *srv, int64_t request_id, double *u, igamg_request_info *info);

/* Snapshot: queued and running requests, completed count, reserved and peak
 * reserved bytes of the budget. */
int igamg_server_status(igamg_server *srv, int *queued, int *running, int64_t *completed,
                        size_t *reserved_bytes, size_t *peak_reserved_bytes);

/* Finish every queued request, stop the workers, free the budget. */
int igamg_server_destroy(igamg_server *srv);
const char *igamg_strerror(int code);
const char *igamg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IGAMG_H */
