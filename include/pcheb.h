/*
 * pcheb — Newton-Chebyshev polynomial-preconditioned conjugate gradients on
 * AMD MI355X (gfx950).
 *
 * The preconditioner is the degree-k polynomial p_k(A) that solves the
 * Chebyshev min-max problem on an interval [alpha, beta] enclosing the spectrum
 * of the Jacobi-scaled operator A = D^-1/2 A_hat D^-1/2 (Bergamaschi &
 * Martinez, arXiv:2008.01440, Sec. 3, eqs. maxmin and cheb).  It is applied
 * with k operator products by the three-term recurrence of Alg. 2, and
 * equals the Newton-based preconditioner of Alg. 1 (Theorem 2).  The
 * "modified parameter" of Sec. 4 multiplies theta = (alpha + beta)/2 by a
 * scale s >= 1 with delta = (beta - alpha)/2 unchanged.
 *
 * Conventions shared by every entry point:
 *  - Pointers named in the argument documentation as "device" must point to
 *    memory on the current HIP device; "host" pointers to host memory.
 *  - Vectors are float64, length n, unit stride.  Several right-hand sides
 *    are stored one after another with leading dimension ld >= n.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL means the null
 *    stream) and is ordered with the caller's other work on that stream.
 *  - No C++ exception crosses this interface.  Every call returns a
 *    pcheb_status; on failure pcheb_last_error() describes the cause.
 *  - A handle may be used by one host thread at a time; distinct handles are
 *    independent.
 */
#ifndef PCHEB_H
#define PCHEB_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pcheb_status {
  PCHEB_OK = 0,
  PCHEB_INVALID = 1,        /* an argument is out of range or inconsistent */
  PCHEB_NOT_SPD = 2,        /* the operator has a non-positive diagonal entry */
  PCHEB_OOM = 3,            /* a device allocation failed */
  PCHEB_HIP = 4,            /* a HIP runtime call failed */
  PCHEB_NOT_CONVERGED = 5,  /* maxit iterations ran without reaching tol */
  PCHEB_BREAKDOWN = 6,      /* (p, Ap) <= 0, (r, z) <= 0, or a non-finite value */
  PCHEB_BUDGET = 7,         /* serving: a request needs more memory than the budget */
  PCHEB_NOT_FOUND = 8,      /* serving: unknown request id */
  PCHEB_PENDING = 9         /* serving: the request has not finished */
} pcheb_status;

typedef enum pcheb_op_kind {
  PCHEB_OP_CSR = 0,         /* general sparse matrix in CSR form */
  PCHEB_OP_SELL = 1,        /* CSR input, stored and streamed as SELL-C-sigma */
  PCHEB_OP_STENCIL7 = 2,    /* matrix-free 7-point Dirichlet Laplacian (diagonal 6, neighbours -1) */
  PCHEB_OP_STENCIL27H = 3   /* matrix-free 27-point harmonic-mean diffusion on cell coefficients */
} pcheb_op_kind;

typedef enum pcheb_precision {
  PCHEB_F64 = 0,            /* p_k(A) recurrence in float64 */
  PCHEB_F32 = 1,            /* matrix values and iterates stored and accumulated in float32 */
  PCHEB_BF16 = 2            /* matrix values and iterates stored in bfloat16, accumulated in float32;
                               degree k <= 32 (see pcheb_setup) */
} pcheb_precision;

/*
 * The unscaled SPD operator A_hat.
 *
 * CSR / SELL: rowptr (int32[n+1]), colind (int32[nnz]) and values
 *   (float64[nnz]) are device arrays in CSR form with nnz < 2^31; they are
 *   borrowed and must stay valid and unchanged until pcheb_destroy.
 *   sell_C must be 0 or 64 (rows per chunk; one wavefront per chunk) and
 *   sell_sigma >= 1 is the row-sorting window (1 keeps the row order).
 * STENCIL7: the 7-point Laplacian on an nx*ny*nz grid, x fastest, with
 *   homogeneous Dirichlet boundaries; n must equal nx*ny*nz.
 * STENCIL27H: cell-centred diffusion on an nx*ny*nz grid, x fastest.
 *   cell_coeff (float64[n], device, borrowed, all in [1e-150, 1e150], else
 *   INVALID; a value <= 0 or not finite is NOT_SPD) holds the cell
 *   coefficients k_i.  Cell i couples to each of its 26 neighbours j with
 *   -H(k_i, k_j), H(a, b) = 2ab/(a + b); a neighbour outside the grid adds
 *   k_i to the diagonal (zero-Dirichlet ghost cell).
 */
typedef struct pcheb_operator {
  int32_t kind;             /* pcheb_op_kind */
  int64_t n;                /* number of unknowns */
  const int32_t* rowptr;    /* CSR/SELL */
  const int32_t* colind;    /* CSR/SELL */
  const double* values;     /* CSR/SELL */
  int64_t nnz;              /* CSR/SELL */
  int32_t nx, ny, nz;       /* stencils */
  const double* cell_coeff; /* STENCIL27H */
  int32_t sell_C;           /* SELL */
  int32_t sell_sigma;       /* SELL */
} pcheb_operator;

/*
 * Preconditioner parameters.  lambda_min < lambda_max bound the spectrum of
 * the Jacobi-scaled operator D^-1/2 A_hat D^-1/2 (Sec. 5 scales every matrix
 * first); lambda_max below the true largest eigenvalue makes p_k(A) A
 * indefinite for odd k.  theta_scale is the modified parameter s of Sec. 4
 * (1 gives the min-max optimal polynomial; the paper uses 1.01 and 1.001).
 * fuse_steps > 1 asks the matrix-free 7-point path to run that many
 * recurrence steps per pass over memory, at most 4 (larger values act as 4;
 * ignored for other operators; 0 or 1 = off).
 * form selects how the same polynomial is applied (Theorem 2 makes them
 * equal in exact arithmetic): PCHEB_FORM_CHEBYSHEV, the three-term
 * recurrence of Alg. 2 (any k); PCHEB_FORM_NEWTON, the recursion of Alg. 1,
 * P_0 u = zeta_0 u, P_{j+1} u = zeta_{j+1} (2 P_j u - P_j A P_j u), which
 * needs k = 2^nlev - 1 (nlev <= 9), F64 or F32 storage (each level evaluates
 * P_j twice, so stored intermediates compound rounding about 2^nlev-fold,
 * too much for BF16) and 2 nlev + 1 extra iterate vectors; it does not fuse
 * steps.
 */
typedef enum pcheb_form {
  PCHEB_FORM_CHEBYSHEV = 0,
  PCHEB_FORM_NEWTON = 1
} pcheb_form;

typedef struct pcheb_params {
  int32_t k;                /* degree = operator products per application, 0 <= k <= 1000 */
  double lambda_min;
  double lambda_max;
  double theta_scale;       /* s >= 1 */
  int32_t prec;             /* pcheb_precision */
  int32_t fuse_steps;
  int32_t form;             /* pcheb_form */
  int32_t block_size;       /* first-level factor P0 = W W^T (closing remark of Sec. 6): 0 or 1 =
                               the Jacobi scaling; 3 = node-block Jacobi (CSR/SELL, n % 3 == 0, the
                               three rows of a node sharing one column pattern): W = blockdiag(L_I^-T)
                               with L_I L_I^T the 3x3 diagonal block of node I, and the polynomial
                               acts on W^T A W (bounds refer to its spectrum) */
  int32_t reserved;         /* 0 */
} pcheb_params;

/* Flags of pcg_solve. */
#define PCG_FLEXIBLE     0x1u  /* Polak-Ribiere beta (z_new, r_new - r_old)/(r_old, z_old) */
#define PCG_X0_GIVEN     0x2u  /* x holds the initial guess; otherwise x0 = 0 */
#define PCG_TIME_KERNELS 0x4u  /* time the middle recurrence steps with HIP events */
#define PCG_NO_GRAPH     0x8u  /* launch each kernel directly instead of replaying HIP graphs */
#define PCG_REFRESH      0x10u /* replace r by b - A x every 50 iterations */

typedef struct pcg_stats {
  int32_t iters;            /* PCG iterations (operator products q = A p) */
  int32_t converged;        /* 1 if recursive ||r|| / ||b|| < tol */
  int32_t status;           /* pcheb_status of the solve */
  int32_t pad0;
  double relres;            /* recursive residual of the scaled system at exit */
  double relres_true;       /* ||b - A x|| / ||b|| of the scaled system, recomputed at exit */
  double relres_true_hat;   /* ||b_hat - A_hat x_hat|| / ||b_hat||, unscaled */
  int64_t n_spmv;           /* operator products, preconditioner included, counted as the
                               textbook loop runs them (a solve that maxit ends counts the
                               application of its last iteration, which the device skips) */
  int64_t n_dot;            /* scalar products, counted as in Table 3 of the paper */
  double seconds;           /* host wall time of the call */
  double step_ms;           /* PCG_TIME_KERNELS: summed time of the middle steps of the
                               applications that did work (one right-hand side, k >= 3) */
  int64_t step_launches;    /* PCG_TIME_KERNELS: number of middle-step launches in step_ms */
} pcg_stats;

typedef struct pcheb_handle_s* pcheb_handle;

/*
 * Build the preconditioner for A_hat (Sec. 3 coefficients, Sec. 4 scaling):
 * computes the diagonal, the recurrence scalars theta' = s (lambda_min +
 * lambda_max)/2, delta = (lambda_max - lambda_min)/2, sigma = theta'/delta,
 * rho_0 = 1/sigma, rho_j = 1/(2 sigma - rho_{j-1}) (eq. rhocheb), the
 * reduced-precision and SELL copies the library owns, and the workspace for
 * one right-hand side.  Synchronises `stream` once.
 * With block_size 3 it also factors the 3x3 diagonal block of every node
 * (second-level preconditioner, see pcheb_params).
 * A bfloat16 recurrence (PCHEB_BF16) is refused above k = 32: the rounding of
 * its stored iterates then costs PCG iterations and moves the solution by more
 * than 1e-6 relative from the float64 recurrence's on 7-point problems.
 * Errors: INVALID (k out of range, BF16 with k > 32, lambda_min <= 0, lambda_min >= lambda_max,
 * s < 1, null or inconsistent arrays, unsupported SELL chunk, block_size not
 * 1 or 3, block_size 3 on a stencil, with n % 3 != 0 or with node rows of
 * different patterns), NOT_SPD (diagonal <= 0, a coefficient <= 0, or a node
 * block that is not positive definite), OOM, HIP.  *out is set only on OK.
 */
pcheb_status pcheb_setup(const pcheb_operator* A, const pcheb_params* p, hipStream_t stream,
                         pcheb_handle* out);

/*
 * z = D^-1/2 p_k(A) D^-1/2 r = p_k(D^-1 A_hat) D^-1 r: the preconditioner for
 * the unscaled system, by Alg. 2 (step j uses rho_j and rho_{j-1}, matching
 * the p_k recurrence of Sec. 3), or by Alg. 1 for the Newton form.  With
 * block_size 3, z = p_k(B^-1 A_hat) B^-1 r with B the node blocks, which is
 * W p_k(W^T A W) W^T r on the scaled system.  r and z are device float64 arrays of
 * nrhs vectors with leading dimension ld; z must not overlap r.  Enqueued on
 * `stream` without host synchronisation.  Errors: INVALID, HIP, OOM.
 */
pcheb_status pcheb_apply(pcheb_handle h, const double* r, double* z, int32_t nrhs, int64_t ld,
                         hipStream_t stream);

/*
 * y = A_hat x in float64 (the unscaled operator; used by the solver for
 * q = A p and by callers to check residuals).  Device arrays, nrhs vectors
 * with leading dimension ld, y must not overlap x.  Errors: INVALID, HIP.
 */
pcheb_status pcheb_matvec(pcheb_handle h, const double* x, double* y, int32_t nrhs, int64_t ld,
                          hipStream_t stream);

/*
 * Solve A_hat x = b by PCG preconditioned with pcheb_apply.  This is PCG on
 * the Jacobi-scaled system of Sec. 5 written in unscaled variables: the
 * iterates are x_hat = D^-1/2 x and the stop test ||r|| / ||b|| < tol uses
 * the D^-1-weighted norm, which is the scaled system's Euclidean norm.
 * b (read) and x (written; read first if PCG_X0_GIVEN) are device float64
 * arrays of nrhs vectors with leading dimension ld.  The outer iteration
 * (residual update, alpha/beta dot products) is float64 whatever the
 * preconditioner precision.  Scalars stay on the device; the host reads
 * them once per group of iterations and at exit, and `stream` is
 * synchronised on return.  stats (host, may be NULL) receives per-solve
 * statistics (nrhs > 1: the slowest right-hand side).
 * Returns OK, NOT_CONVERGED (x holds the last iterate), BREAKDOWN, INVALID,
 * HIP or OOM.
 */
pcheb_status pcg_solve(pcheb_handle h, const double* b, double* x, int32_t nrhs, int64_t ld,
                       double tol, int32_t maxit, uint32_t flags, pcg_stats* stats,
                       hipStream_t stream);

/* Release everything the handle owns (not the borrowed operator arrays).  NULL is allowed. */
pcheb_status pcheb_destroy(pcheb_handle h);

/*
 * Work lists: several problems, each with its own operator and preconditioner,
 * advanced by one launch per kernel for all of them (the Alg. 2 steps and the
 * PCG iteration of every problem; grid dimension z selects the problem).  This
 * is the batched counterpart of pcheb_apply and pcg_solve for many problems of
 * one shape, e.g. one mesh with many coefficient fields: a launch then covers
 * count times the tiles of one problem, which fills the chip where a single
 * small problem cannot, and a PCG iteration costs the launches of one problem.
 *
 * The handles must describe problems whose launches coincide: the same
 * operator kind and shape (stencil grid; CSR/SELL n, row-length class and
 * chunking), precision, degree k, form and steps per pass.  Their operator
 * data, spectral bounds (so the recurrence coefficients) and 27-point
 * coefficient fields may all differ.  pcheb_group_create checks this by
 * comparing the launches each handle would make and fails with INVALID,
 * naming the first difference, otherwise.
 * Each problem's result equals, bit for bit, that of the same call on its
 * own handle: every block does the work it does in that handle's own launch.
 * The group borrows the handles (count in [1, 1024], no duplicates); they must
 * outlive it.  Group calls use the handles' workspaces: work enqueued with a
 * handle on another stream must not overlap a group call's work (order the
 * streams, as for two calls on one handle).  A group call first waits on the
 * host until the device has finished the previous call of the same group (its
 * argument tables are rewritten).  Every device block comes from the allocator
 * of pcheb_set_allocator when one is installed.
 * Errors: INVALID, OOM, HIP.  *out is set only on OK.
 */
typedef struct pcheb_group_s* pcheb_group;
pcheb_status pcheb_group_create(const pcheb_handle* handles, int32_t count, pcheb_group* out);

/*
 * z_i = P_k(i) r_i for every problem i of the group (pcheb_apply with nrhs 1
 * on each handle): r and z are device float64 arrays of `count` vectors with
 * leading dimension ld (vector i at offset i ld), 16-byte aligned, z not
 * overlapping r.  Enqueued on `stream` without host synchronisation.
 * Errors: INVALID, HIP, OOM.
 */
pcheb_status pcheb_group_apply(pcheb_group g, const double* r, double* z, int64_t ld, hipStream_t stream);

/*
 * pcg_solve of every problem i of the group on (b_i, x_i), the vectors at
 * offset i ld of the device float64 arrays b and x, all with the same tol,
 * maxit and flags (PCG_FLEXIBLE, PCG_X0_GIVEN, PCG_NO_GRAPH; PCG_TIME_KERNELS
 * and PCG_REFRESH are INVALID here).  Problems converge independently; the
 * launches skip the finished ones.  stats (host, may be NULL) receives `count`
 * entries, one per problem.  `stream` is synchronised on return.
 * Returns OK if every problem converged, else the status of the first that
 * did not (NOT_CONVERGED or BREAKDOWN), or INVALID, HIP, OOM.
 */
pcheb_status pcg_solve_group(pcheb_group g, const double* b, double* x, int64_t ld, double tol,
                             int32_t maxit, uint32_t flags, pcg_stats* stats, hipStream_t stream);

/* Release the group's tables and graphs (not its handles).  NULL is allowed. */
pcheb_status pcheb_group_destroy(pcheb_group g);

/* Description of the last failure on the calling thread ("" if none).  Valid until the next call. */
const char* pcheb_last_error(void);

/* Device bytes pcheb_setup plus pcg_solve with nrhs right-hand sides will allocate. */
size_t pcheb_footprint_bytes(const pcheb_operator* A, const pcheb_params* p, int32_t nrhs);

/*
 * Device memory.  Every block of device memory the library allocates (a
 * handle's operator copies and solve workspace, the bound estimators'
 * workspace, the server's resident groups, right-hand-side and solution
 * staging and Lanczos start vectors) comes from alloc_fn once it is installed,
 * so a caller's pool (for example PyTorch's caching allocator) supplies it;
 * the problem statement of Sec. 1 leaves memory to the caller's environment.
 *  - alloc_fn(bytes, ctx) returns a block of at least `bytes` bytes on the
 *    current device, 256-byte aligned and usable from any stream, or NULL (the
 *    library call then fails with PCHEB_OOM).  It may be called from any host
 *    thread, including the server's own threads, with that device current.
 *  - free_fn(ptr, bytes, ctx) takes a block back.  The library calls it only
 *    once no device work that may use the block is pending (it synchronises the
 *    device first when a handle, an estimate or a server group releases
 *    memory), and always with the free_fn and ctx that were installed when the
 *    block was allocated, even if another allocator has been installed since.
 *  - Both NULL restores hipMalloc / hipFree for later allocations.  The
 *    setting is process-wide and is read at each allocation.
 * Not covered: the small pinned host mirrors of solver states
 * (hipHostMalloc) and memory the HIP runtime allocates for itself (graphs,
 * the fixed scratch array of pcheb_estimate_bounds_noalloc).
 * Errors: INVALID if exactly one of the two functions is NULL.
 */
typedef void* (*pcheb_alloc_fn)(size_t bytes, void* ctx);
typedef void (*pcheb_free_fn)(void* ptr, size_t bytes, void* ctx);
pcheb_status pcheb_set_allocator(pcheb_alloc_fn alloc_fn, pcheb_free_fn free_fn, void* ctx);

/*
 * Extreme Ritz values of nsteps Lanczos steps (classical Gram-Schmidt
 * against all previous vectors, twice) on the Jacobi-scaled operator
 * D^-1/2 A_hat D^-1/2, started from v0 (device float64[n], 16-byte aligned,
 * need not be normalised).  The tridiagonal stops at the first beta_j that
 * vanishes relative to alpha_j (exhausted Krylov space).  The paper
 * estimates the bounds by the power method and DACG (Sec. 5.1); callers
 * widen lambda_max by a safety factor before pcheb_setup.  Writes
 * *lambda_min, *lambda_max (host); synchronises `stream` before returning.
 * Allocates nsteps + 4 vectors of workspace for the duration of the call.
 * Errors: INVALID (also a zero or non-finite v0), NOT_SPD, OOM, HIP.
 */
pcheb_status pcheb_estimate_bounds(const pcheb_operator* A, const double* v0, int32_t nsteps,
                                   double* lambda_min, double* lambda_max, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture
 * around the call, tight serving loops, harnesses that forbid hipMalloc):
 * pcheb_estimate_bounds, with the same arguments, results (bit for bit) and
 * errors, that allocates nothing.  Its workspace - the Lanczos basis, the
 * vectors, the operator's diagonal and the reduction partials - lives in a
 * fixed device array of PCHEB_NOALLOC_SCRATCH_BYTES that the library holds on
 * every device it has run this call on, until the process ends; the call
 * takes it over without clearing it first (nothing in it is read before it is
 * written).  The workspace is
 *   8 * ((nsteps + 1) * round_up(n, 2) + (2 + d) * n + 3 * nsteps + 3) + 524288
 * bytes plus at most 2 KiB of alignment, with d = 0 for STENCIL7, 1 for CSR or
 * SELL and 2 for STENCIL27H (nsteps capped at n): with 30 steps, up to about
 * 500,000 unknowns of a 7-point grid (79^3).  A larger operator returns INVALID before
 * any work is enqueued.  Every call on a device uses that device's one array:
 * calls that overlap on one GPU (from two host threads, or on two streams
 * without ordering between them) race and give wrong results.  Synchronises
 * `stream` as pcheb_estimate_bounds does.
 */
#define PCHEB_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
pcheb_status pcheb_estimate_bounds_noalloc(const pcheb_operator* A, const double* v0, int32_t nsteps,
                                           double* lambda_min, double* lambda_max, hipStream_t stream);

/*
 * As pcheb_estimate_bounds, for the operator the preconditioner with first-level
 * block size `block_size` acts on: 1 gives D^-1/2 A_hat D^-1/2 (the same as
 * pcheb_estimate_bounds); 3 gives W^T A W on the node-block Jacobi factor of
 * the Jacobi-scaled A (pcheb_params.block_size), that is L^-1 A_hat L^-T with
 * L L^T the 3x3 diagonal blocks of A_hat (CSR/SELL, n % 3 == 0).  Allocates
 * nsteps + 5 vectors for the duration of the call.  Errors as
 * pcheb_estimate_bounds; INVALID also for another block size or a node whose
 * rows differ in pattern, NOT_SPD for a block that is not positive definite.
 */
pcheb_status pcheb_estimate_bounds_block(const pcheb_operator* A, int32_t block_size, const double* v0,
                                         int32_t nsteps, double* lambda_min, double* lambda_max,
                                         hipStream_t stream);

/*
 * The paper's bound estimates (Sec. 5.1) for the Jacobi-scaled operator
 * A = D^-1/2 A_hat D^-1/2, both started from v0 (device float64[n], need not
 * be normalised; it is only read):
 *  - lambda_max: power_iters steps of the power method, v <- A v / ||A v||;
 *    the Rayleigh quotient of the last iterate (a lower estimate of
 *    lambda_max: callers widen it before pcheb_setup);
 *  - lambda_min: the DACG method without preconditioning (conjugate-gradient
 *    minimisation of the Rayleigh quotient, Bergamaschi, Gambolati and Pini
 *    1997) until ||A x - mu x|| / (mu ||x||) <= dacg_tol (the paper uses
 *    1e-2) or dacg_maxit steps; mu is an upper estimate of lambda_min.
 * Writes *lambda_min, *lambda_max and, if not NULL, *dacg_steps and
 * *dacg_relres (host); synchronises `stream` before returning.  Allocates 6
 * vectors of workspace for the duration of the call.  One operator product
 * per power step and per DACG step.
 * Errors: INVALID (bad arguments, a zero or non-finite v0), NOT_SPD,
 * BREAKDOWN (non-finite values, or a direction parallel to the iterate),
 * OOM, HIP.  Reaching dacg_maxit is not an error: *dacg_relres tells.
 */
pcheb_status pcheb_estimate_bounds_pdacg(const pcheb_operator* A, const double* v0, int32_t power_iters,
                                         double dacg_tol, int32_t dacg_maxit, double* lambda_min,
                                         double* lambda_max, int32_t* dacg_steps, double* dacg_relres,
                                         hipStream_t stream);

/* Seeded uniform vector (workload generation, not part of the method):
 * v[i] = lo + (hi - lo) * U_i for i < n, where U_i is element i of the
 * counter-based SplitMix64 stream of `seed` (Steele, Lea & Flood, OOPSLA
 * 2014): mix(seed + (i + 1) * 0x9E3779B97F4A7C15) with the SplitMix64
 * finaliser, top 53 bits times 2^-53.  Bitwise equal to a sequential
 * implementation of the same definition.  v: device float64[n], caller-owned.
 * Stream-ordered, no host sync.  Errors: INVALID (n < 0, null v, lo > hi), HIP.
 */
pcheb_status pcheb_fill_uniform(double* v, int64_t n, uint64_t seed, double lo, double hi, hipStream_t stream);

/* ------------------------------------------------------------------ serving
 *
 * A solve server with continuous batching.  Requests (an operator, a degree,
 * a precision, a tolerance and a right-hand side) are admitted as long as
 * the device memory they need fits the budget; requests with the same
 * operator and parameters share one resident preconditioner (operator data,
 * eigenvalue bounds, workspace for max_nrhs right-hand sides) and iterate
 * together in multi-vector launches replayed from HIP graphs, each with its
 * own scalars and stop test.  Requests join a running group between groups
 * of iterations as slots free up, leave it when they converge, and groups of
 * different operators run concurrently on their own streams.  A request's
 * result does not depend on what else is being solved (same launches and
 * reduction order per right-hand side).
 *
 * Every request iterates with the flexible (Polak-Ribiere) beta, so results
 * equal those of pcg_solve with PCG_FLEXIBLE, x0 = 0, on the same parameters.
 * Memory counted against the budget: pcheb_footprint_bytes(op, params,
 * max_nrhs) plus 2 * max_nrhs * round_up(n, 64) doubles of right-hand-side
 * and solution staging per resident group; a bound estimate borrows its
 * Lanczos vectors for the duration of the group set-up only.
 *
 * One host thread owned by the server does all device work; the calls below
 * may be made from any thread, except pserve_destroy, which must not race
 * with the others.  A finished request's id is released once pserve_poll has
 * reported it done or pserve_wait has returned; later calls with that id
 * return NOT_FOUND.  Cancelling a request that is already finishing has no
 * effect.
 */
typedef struct pserve_s* pserve_handle;

typedef struct pserve_request {
  pcheb_operator op;    /* device arrays borrowed until the request completes */
  int32_t k;            /* degree */
  int32_t prec;         /* pcheb_precision */
  double lambda_min;    /* bounds of the scaled operator; lambda_max <= 0: estimate them */
  double lambda_max;    /*   (30 Lanczos steps, lambda_max widened by 1.01; once per operator) */
  double theta_scale;   /* modified parameter s >= 1 */
  double tol;           /* relative residual tolerance */
  int32_t maxit;
  int32_t fuse_steps;
  const double* b;      /* device float64[n], ready when submitted (the server reads it on its own
                           stream, unordered with the caller's); read-only until the request completes */
  double* x;            /* device float64[n]; receives the solution; complete when the request is
                           reported done */
  uint64_t op_key;      /* requests with equal op_key and equal operator fields share resident data */
} pserve_request;

typedef struct pserve_stats {
  int64_t submitted, admitted, completed, rejected, cancelled;
  int64_t queued, active;           /* now */
  int64_t groups, groups_created, groups_evicted;
  int64_t bytes_in_use, bytes_high_water, budget;
  int64_t launches;                 /* iteration-group launches */
  int64_t batch_hist[8];            /* launches with 1, 2, 3-4, 5-8, 9-16, 17-32, 33-64, >64 active solves */
} pserve_stats;

/* Create a server with a device-memory budget (bytes) and at most max_nrhs
 * concurrent solves per resident operator (1..64), on the current device. */
pcheb_status pserve_create(size_t hbm_budget, int32_t max_nrhs, pserve_handle* out);

/* Queue a request; *id identifies it.  Returns BUDGET if the request alone
 * needs more memory than the budget, INVALID for bad arguments. */
pcheb_status pserve_submit(pserve_handle srv, const pserve_request* req, uint64_t* id);

/* *done = 1 and stats filled once the request has finished (stats->seconds is
 * the latency from submission to completion; stats->status its final status,
 * with the reason in pcheb_last_error() when it is not OK), else *done = 0.
 * NOT_FOUND for unknown ids. */
pcheb_status pserve_poll(pserve_handle srv, uint64_t id, int32_t* done, pcg_stats* stats);

/* Block until the request has finished; returns its solve status (OK,
 * NOT_CONVERGED, BREAKDOWN; NOT_CONVERGED for a cancelled request), or the
 * error that ended it (e.g. INVALID or NOT_SPD from the set-up of its
 * operator, OOM). */
pcheb_status pserve_wait(pserve_handle srv, uint64_t id, pcg_stats* stats);

/* Drop a queued or running request; its slot is freed, others are unaffected. */
pcheb_status pserve_cancel(pserve_handle srv, uint64_t id);

pcheb_status pserve_get_stats(pserve_handle srv, pserve_stats* out);

/* Stop the server (running requests are dropped) and free everything. */
pcheb_status pserve_destroy(pserve_handle srv);

#ifdef __cplusplus
}
#endif

#endif /* PCHEB_H */
