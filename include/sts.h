/*
 * sts.h -- space-time Sylvester solver for the heat equation on one MI355X.
 *
 * Solves the space-time Petrov-Galerkin system of the heat equation
 * (hat functions in time for trial, indicators in time for test, P1/Q1
 * elements in space; Sec. 3 of Henning, Palitta, Simoncini, Urban,
 * "Matrix oriented reduction of space-time Petrov-Galerkin variational
 * problems", eq. (par1)-(par2)) in its matrix form, the generalized
 * Sylvester equation of Sec. 4, eq. (Sylv_Heat):
 *
 *     Kx U Mt^T + Mx U Dt^T = F1 F2^T,      U in R^{Nh x Nt},
 *
 * where Kx = mu * stiffness, Mx = mass (Nh x Nh, SPD), Dt[l,k] =
 * (d/dt sigma^k, tau^l), Mt[l,k] = (sigma^k, tau^l) (Nt x Nt, lower
 * bidiagonal, indexed [test l, trial k]) and F1 (Nh x P), F2 (Nt x P) are the
 * factors of the low-rank load (Sec. 3, eq. (EIM)).  Column l-1 of U holds the
 * nodal values at time t^l; u(t^0) = 0 is not stored.
 *
 * The solver is the Galerkin projection of Sec. 4: the spatial space is grown
 * as an extended Krylov space (rational Krylov with the poles 0 and infinity)
 * in the operator Mx^{-1} Kx started from Mx^{-1} F1; the basis V is
 * orthonormal in the Mx inner product; the reduced equation
 * (V^T Kx V) Y Mt^T + (V^T Mx V) Y Dt^T = (V^T F1) F2^T is solved by
 * diagonalising the reduced spatial pencil and sweeping the bidiagonal time
 * recurrence per eigencomponent; the residual is monitored in projected form
 * and confirmed by the exact residual before success is reported.  The result
 * is returned as the factors V (Nh x k) and Y (k x Nt), U ~= V Y.
 *
 * Conventions (all entry points)
 *   - Column-major storage, leading dimensions in elements, FP64 throughout.
 *   - Grid nodes are the interior nodes of a uniform grid on the unit
 *     interval / square / cube, numbered lexicographically with x fastest.
 *   - Pointers marked "device" must be device memory of the current HIP
 *     device; "host" means host memory; "mem" arguments select between them
 *     (STS_MEM_HOST / STS_MEM_DEVICE).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work of a call is ordered on that stream.  Calls marked
 *     "synchronous" wait for their own work before returning.
 *   - Every function returns an sts_status; none throws or aborts.  On error
 *     sts_last_error() returns a description (thread-local, valid until the
 *     next call on the same thread).
 *   - The library allocates its own device memory with hipMalloc and frees it
 *     in sts_destroy (or before returning, for the step-level calls).  It
 *     never frees caller memory.
 */
#ifndef STS_H
#define STS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STS_OK = 0,
  STS_E_INVALID = 1,       /* bad argument: sizes, strides, NULL, non-finite data */
  STS_E_NOMEM = 2,         /* device allocation failed or exceeds the memory budget */
  STS_E_DEVICE = 3,        /* a HIP runtime call failed */
  STS_E_NOT_CONVERGED = 4, /* max_outer reached; factors of the last iterate stay fetchable */
  STS_E_NUMERIC = 5,       /* breakdown: CG curvature <= 0, NaN/Inf, basis lost orthogonality */
  STS_E_STATE = 6          /* call out of order (e.g. get_factors before solve) */
} sts_status;

typedef enum { STS_MEM_HOST = 0, STS_MEM_DEVICE = 1 } sts_mem;

/* Spatial discretisation (Sec. 3: conforming X_h; P1 elements).
 *   STS_FE_P1_1D       (0,1), P1 hats: Kx = (mu/h) tridiag(-1,2,-1),
 *                      Mx = (h/6) tridiag(1,4,1).
 *   STS_FE_P1_2D       unit square, P1 on the uniform Courant triangulation
 *                      (squares cut along the SW-NE diagonal): Kx = mu *
 *                      5-point (4; -1), Mx = (h^2/12)(6; 1 at E,W,N,S,NE,SW).
 *   STS_FE_Q1_3D_7PT   unit cube, trilinear elements: consistent Q1 mass
 *                      (27-point, the tensor product of 1-D P1 masses) and the
 *                      Q1 stiffness with lumped transverse mass (7-point,
 *                      mu h (6; -1 on faces)).
 * n[d] = interior nodes in direction d (n[d] = 1 for unused directions),
 * h = 1/(n[d]+1) (the grid must be isotropic: equal n[d] for used d). */
typedef enum { STS_FE_P1_1D = 1, STS_FE_P1_2D = 2, STS_FE_Q1_3D_7PT = 3 } sts_fe_kind;

typedef struct {
  int32_t kind;   /* sts_fe_kind */
  int32_t pad_;
  int64_t n[3];   /* interior nodes per direction */
  double mu;      /* diffusion coefficient (> 0) */
} sts_space;

/* Which spatial operator a step-level call applies. */
typedef enum { STS_OP_K = 0, STS_OP_M = 1 } sts_op;

/* Lower-bidiagonal Nt x Nt time matrix: diag[l] = A[l,l] (length nt),
 * sub[l] = A[l+1,l] (length nt-1).  Host pointers. */
typedef struct {
  const double* diag;
  const double* sub;
} sts_bidiag;

typedef struct {
  double tol;               /* relative Frobenius residual target (Sec. 5 uses 1e-8); default 1e-8 */
  int32_t max_outer;        /* max extended-Krylov blocks; default 200 */
  int32_t check_every;      /* 0 = adaptive residual checks, n > 0 = every n blocks; default 0 */
  double inner_rtol;        /* CG relative residual target; default 1e-13 */
  int32_t inner_maxit;      /* CG iteration cap per solve; default 200000 */
  int32_t verify_true;      /* 1 = confirm convergence with the exact residual; default 1 */
  double defl_tol;          /* drop a new column whose Mx-norm falls below this fraction; default 1e-10 */
  int64_t mem_budget;       /* bytes of device memory the problem may hold; 0 = unlimited */
  int32_t restart;          /* 1 = discard the current basis and solve from scratch; default 0 */
  int32_t profile;          /* 1 = time the main kernels with HIP events (sts_kernel_profile);
                               default 0 */
  int32_t inner_precond;    /* 1 = fast inner solvers where the space allows them: 1-D P1,
                               Kx and Mx by a direct tridiagonal solve; 2-D P1 with n <= 63
                               or n odd halving, n -> (n-1)/2, down to <= 255: Kx by CG
                               preconditioned with one geometric multigrid V-cycle, Mx by
                               Chebyshev iteration; 3-D trilinear: Mx by direct line solves,
                               Kx by multigrid-preconditioned CG when n <= 63 or n odd halving
                               down to <= 63 (else plain CG); 0 = plain CG for both; default 1 */
  int32_t rational;         /* projection space: 0 = extended Krylov (poles 0 and infinity);
                               1 = rational Krylov with adaptive shifts (Sec. 4): after the
                               extended start block, each step applies (Kx + s Mx)^{-1} Mx to
                               the last block, s chosen by the greedy rule of
                               sts_adaptive_shift from the Ritz values; convergence is
                               checked on the exact residual; default 0 */
  int32_t residual_qr;      /* exact residual ||A B^T|| (A = [F1, Kx V, Mx V], B its time
                               factor, Nt x (P + 2k)): 1 = through the Householder QR of B,
                               ||A R_B^T||, whenever 2 (P + 2k) <= Nt <= 4096; -1 = always the
                               direct Nh x Nt product; 0 = the cheaper of the two by a cost
                               model; default 0 */
  int32_t inner_relax;      /* j = 1..6: relax the inner tolerance as the residual falls
                               (inexact Krylov): the inner solves of each block stop at
                               max(inner_rtol, min(1e-4, 10^-j tol / r)), r the last projected
                               residual estimate (1 before the first check); the exact residual
                               still decides convergence; 0 = inner_rtol throughout; default 0 */
  int32_t precond_fp32;     /* 1 = mixed precision in the 3-D Kx solves (and the shifted solves
                               of the rational Krylov space): the multigrid V-cycle that
                               preconditions CG stores its vectors in FP32 (arithmetic in FP64);
                               CG itself, its residuals, iterates and stopping test stay FP64, so
                               the solves reach the same tolerances.  Applies to 3-D seven-point
                               spaces with n > 63 (at least one smoothed level); elsewhere
                               ignored.  0 = FP64 throughout; default 0 */
  int32_t mixed;            /* 1 = FP32 bulk with FP64 refinement: the 3-D Kx solves run
                               multigrid PCG in FP32 (every vector, the stencil product, the
                               V-cycle, per-tile inner products) inside FP64 defect correction
                               (x += d, r = b - Kx x in FP64 until ||r|| <= rtol ||b||, FP64 PCG
                               finishing a column whose FP32 rounds stall), and the first
                               classical Gram-Schmidt pass takes its coefficients from an FP32
                               copy of V with FP32 accumulation (the update uses the FP64 basis,
                               so each block stays in the span of the expansion); the second
                               (re-orthogonalisation) pass, the reduced
                               matrices, eigensolve, time sweep and the exact Sylvester
                               residual that decides convergence stay FP64.  Applies to 3-D
                               seven-point spaces with n > 63; elsewhere ignored.  Takes
                               precedence over precond_fp32 in the FP32 rounds.  2 = the FP32
                               Kx solves only, 3 = the FP32 Gram-Schmidt pass only (the two
                               parts apart); 0 = FP64 throughout; default 0 */
  int32_t orth_lag;         /* 1 = lagged re-orthogonalisation of the Mx Gram-Schmidt of the
                               basis (Sec. 4's orthonormal columns; the block form of the delayed
                               second pass of classical Gram-Schmidt run twice): a new block is
                               orthogonalised once and normalised provisionally, the next block
                               is expanded from it, and its second pass comes with the next
                               block's first in the same two reads of the basis, halving the
                               reads per block; blocks before a residual check get both passes
                               at once.  Not used in the rational space, with the FP32 first
                               pass (mixed 1 or 3), or in 1-D (small bases, kappa(Mx^-1 Kx) up
                               to 1e10).  0 = both passes per block; default 1 */
  int32_t pad_;             /* zero */
} sts_opts;

typedef struct {
  int32_t outer_its;        /* blocks added after the start block */
  int32_t checks;           /* reduced solves performed */
  int64_t k;                /* basis size of the returned factors (mu_mem of Sec. 5, Table 1) */
  int64_t rank;             /* numerical rank of V Y (singular values > 1e-8 sigma_1) */
  int64_t inner_its_K;      /* CG iterations on Kx, summed over columns and solves */
  int64_t inner_its_M;      /* CG iterations on Mx, summed over columns and solves */
  double res_cheap;         /* last projected residual estimate (relative Frobenius) */
  double res_true;          /* exact relative residual of the returned factors, or -1 */
  double orth_err;          /* max |V^T Mx V - I| over the reduced matrix */
  double seconds;           /* wall time of sts_solve */
  double alg_bytes;         /* algorithmic HBM bytes moved by the kernels (model) */
  int32_t breakdown;        /* 1 = the space became invariant (exact solution) */
  int32_t shifts;           /* shifted solves of a rational Krylov space (0 otherwise) */
  int64_t cg_poll_restarts; /* times a polled CG state was stale and iterations resumed */
  double res_floor;         /* estimated rounding floor of the exact residual in FP64 (see
                               sts_solve), or -1 where it was not needed */
  int32_t floor_limited;    /* 1 = accepted with res_true above tol, within the rounding floor
                               (sts_solve) */
  int32_t pad_;
  int64_t inner_its_fp32;   /* FP32 PCG iterations of the mixed-precision Kx solves (included
                               in inner_its_K) */
  int64_t defect_rounds;    /* FP64 defect corrections of the mixed-precision Kx solves */
} sts_info;

/* Kernels timed by sts_kernel_profile. */
typedef enum {
  STS_K_CG_ITER = 0,        /* plain CG iteration (stencil SpMM + vector updates) */
  STS_K_MG_DOWN = 1,        /* multigrid: smoothing, residual, restriction */
  STS_K_MG_UP = 2,          /* multigrid: prolongation and smoothing */
  STS_K_MG_COARSE = 3,      /* multigrid: exact coarsest-level solve */
  STS_K_PCG_A = 4,          /* preconditioned CG: direction and K p */
  STS_K_PCG_B = 5,          /* preconditioned CG: x and r updates */
  STS_K_MASS_CHEB = 6,      /* Chebyshev steps of an Mx solve */
  STS_K_GRAM = 7,           /* Gram contraction V^T W (matrix cores) */
  STS_K_BASIS_UPDATE = 8,   /* W -= V C (matrix cores) */
  STS_K_RESIDUAL = 9,       /* exact residual norm (matrix cores) */
  STS_K_TRIDIAG = 10,       /* reduced eigensolve: tridiagonalisation */
  STS_K_BISECT = 11,        /* reduced eigensolve: eigenvalues */
  STS_K_INVITER = 12,       /* reduced eigensolve: eigenvectors of T */
  STS_K_BACKTRANSFORM = 13, /* reduced eigensolve: back-transformation */
  STS_K_SWEEP = 14,         /* time sweep */
  STS_K_STENCIL = 15,       /* stencil SpMM Kx V, Mx V */
  STS_K_TRIDIAG_SOLVE = 16, /* direct tridiagonal inner solve (1-D) */
  STS_K_MG_RESTRICT = 17,   /* multigrid (3-D): residual and restriction */
  STS_K_PCG_REDUCE = 18,    /* preconditioned CG (3-D): sums of per-tile partials */
  STS_K_RESIDUAL_QR = 19,   /* Householder QR of the residual's time factor */
  STS_K_GRAM_REDUCE = 20,   /* sum of the Gram contraction's per-chunk partial products */
  STS_K_COUNT = 21
} sts_kernel;

typedef struct sts_problem sts_problem;

/* Fill *o with the defaults listed in sts_opts. */
void sts_default_opts(sts_opts* o);

/* Time matrices of the hat/indicator pair (Sec. 3, eq. (par1)) on the nodes
 * t[0..nt] (host, strictly increasing): Dt diag = 1, sub = -1; Mt diag =
 * sub = (t[l+1]-t[l])/2 on row l.  Outputs are host arrays (nt and nt-1). */
sts_status sts_time_matrices(int64_t nt, const double* t, double* dt_diag, double* dt_sub,
                             double* mt_diag, double* mt_sub);

/* Create a problem: the generalized Sylvester equation of Sec. 4, eq.
 * (Sylv_Heat), Kx U Mt^T + Mx U Dt^T = F1 F2^T, for the space-time
 * discretisation of Sec. 3 (eq. (par1)-(par2)) with a low-rank load F1 F2^T
 * (Sec. 3, eq. (EIM)).  The spatial matrices are not passed: Kx and Mx are the
 * matrix-free stencils of the built-in space kinds (sts_fe_kind), so a caller
 * cannot supply its own sparse matrices.  Dt, Mt are host lower bidiagonals
 * (any strictly positive diagonals: uniform or graded time steps).  Copies F1
 * (Nh x p, ld ldf1) and F2 (nt x p, ld ldf2) from `mem` into library memory;
 * the caller keeps its arrays.  Errors: STS_E_INVALID for nt < 2, p < 1 or
 * p > 4, ld < rows, non-positive diagonals of Dt or Mt, non-finite data or an
 * unsupported space; STS_E_NOMEM / STS_E_DEVICE on allocation or copy
 * failure.  Synchronous. */
sts_status sts_create(const sts_space* space, const sts_bidiag* Dt, const sts_bidiag* Mt,
                      int64_t nt, int32_t p, const double* F1, int64_t ldf1,
                      const double* F2, int64_t ldf2, int32_t mem, void* stream,
                      sts_problem** out);

/* Solve to opts->tol (NULL = defaults) by the Galerkin projection of Sec. 4:
 * grow the spatial space block by block, solve the reduced equation
 * (V^T Kx V) Y Mt^T + (V^T Mx V) Y Dt^T = (V^T F1) F2^T, and stop on the
 * relative residual R_m of Sec. 4 (Sec. 5 uses 1e-8).  Fills *info if
 * non-NULL.  May be called again on the same problem with a tighter tolerance:
 * the space is extended from where the previous call stopped.
 *
 * Device memory: V, Mx V and Kx V (Nh x k each) grow with the space, 16p
 * columns at a time and to at most max_outer + 2 more blocks, by
 * reallocation and a device copy (old and new copies of one array coexist
 * for that moment), so the problem holds what the basis uses, not what
 * max_outer allows.  opts->mem_budget bounds the total.
 *
 * Convergence is decided by the projected residual and confirmed by the
 * exact one (opts->verify_true).  The exact residual is evaluated from the
 * solution stored in FP64, which rounds U's entries; that alone moves the
 * residual by about u kappa(Mx^{-1} Kx) relative to F (u = 2^-53; about 1e-7
 * for the 1-D problem with 65535 nodes, where no FP64 representation of the
 * exact solution has a smaller residual).  When the projected residual meets
 * tol but the exact one does not, the library estimates that floor
 * (info->res_floor); if it is at least tol / 2 and the exact residual lies
 * within tol + floor, the solve is accepted (info->floor_limited = 1).  The
 * floor grows like sqrt(k / 64) beyond 64 basis columns (the backward error
 * of the order-k reduced eigendecomposition).  Where the estimated floor
 * alone exceeds tol, the projected residual is driven to tol + floor instead
 * of tol.  Where the floor is at least tol / 2 the inner solves carry the
 * same rounding, and the projected residual itself can stall above tol: a
 * solve whose projected residual has not halved over three checks is
 * accepted with an exact residual within tol + 4 floor (floor_limited = 1),
 * else it continues.
 *
 * Returns STS_OK; STS_E_NOT_CONVERGED when max_outer blocks did not reach tol
 * (the factors of the last iterate are kept and fetchable); STS_E_NUMERIC on a
 * breakdown -- a non-positive curvature or non-finite value in an inner solve,
 * a non-finite reduced matrix, or a block whose every column deflated while
 * the exact residual is still above tol (the factors are kept); STS_E_NOMEM.
 * A block that deflates entirely with the exact residual at tol is the
 * invariant-space case: STS_OK with info->breakdown = 1.  Synchronous. */
sts_status sts_solve(sts_problem* prob, const sts_opts* opts, sts_info* info);

/* Number of columns of V (rows of Y) of the current solution U ~= V Y:
 * the basis size mu_mem that Sec. 5, Table 1 reports. */
sts_status sts_rank(const sts_problem* prob, int64_t* k);

/* Columns of the low-rank solution U ~= V Y of Sec. 4 at chosen time steps
 * without copying V: U[:, j] = V Y[:, cols[j]] for j < ncols, computed on the
 * device (the nodal values at time t^{cols[j] + 1}).  cols (host, ncols >= 1
 * entries in 0..nt-1); U (Nh x ncols, ldu >= Nh) in host or device memory as
 * `mem` says.  STS_E_STATE before a solve, STS_E_INVALID for bad indices or
 * buffers.  Synchronous. */
sts_status sts_solution_columns(const sts_problem* prob, const int64_t* cols, int32_t ncols,
                                double* U, int64_t ldu, int32_t mem, void* stream);

/* Copy the factors of the low-rank solution U ~= V Y of Sec. 4 (V the
 * Mx-orthonormal spatial basis, Y the reduced solution) into caller buffers:
 * V (Nh x k, ld ldv >= Nh) and Y (k x nt, ld ldy >= k), either may be NULL;
 * `mem` says whether the buffers are host or device memory.  The library
 * keeps its copies.  STS_E_STATE before a successful or not-converged solve.
 * Synchronous. */
sts_status sts_get_factors(const sts_problem* prob, double* V, int64_t ldv, double* Y,
                           int64_t ldy, int32_t mem, void* stream);

/* Exact relative residual ||F1 F2^T - Kx V Y Mt^T - Mx V Y Dt^T||_F / ||F1 F2^T||_F
 * of the current factors (Sec. 4, residual R_m).  Synchronous. */
sts_status sts_true_residual(sts_problem* prob, double* res);

/* Numerical rank of the current solution V Y (Sec. 5 reports rank(U)): the
 * number of singular values of V Y in the Mx norm (those of Y, V being
 * Mx-orthonormal) above 1e-8 times the largest.  Synchronous. */
sts_status sts_numerical_rank(sts_problem* prob, int64_t* rank);

/* Kernel timing of the last sts_solve made with opts.profile = 1: summed
 * event time (seconds) of the launches of `kernel` (sts_kernel), their count
 * and their algorithmic bytes (the data the operation must read and write
 * once, in the model stated beside each kernel in the sources).  Outputs are
 * host pointers, each may be NULL.  STS_E_STATE if that solve did not
 * profile.  Synchronous (waits for the events). */
sts_status sts_kernel_profile(sts_problem* prob, int32_t kernel, double* seconds,
                              int64_t* launches, double* alg_bytes);

/* Short name of an sts_kernel ("" if out of range). */
const char* sts_kernel_name(int32_t kernel);

/* Free everything the problem holds.  NULL-safe.  Device blocks of 16 MiB and
 * more go to the library's block cache (kept per device, up to 32 GiB idle,
 * for later problems of similar size; reusing a block avoids seconds of
 * driver work at gigabyte sizes), the rest back to the driver. */
void sts_destroy(sts_problem* prob);

/* Return every idle block of the library's cache to the driver (e.g. before
 * another allocator on the same GPU needs the memory); blocks held by live
 * problems are not affected.  A failed allocation inside the library does
 * this by itself before it reports STS_E_NOMEM.  Thread-safe. */
void sts_release_cached_memory(void);

/* Description of the last error on this thread ("" if none). */
const char* sts_last_error(void);

/* ------------------------------------------------------------------------
 * Step-level entry points (each runs one step of the solver's path on
 * caller-provided device buffers; used for parity checks).  All pointers are
 * device pointers; scratch is allocated and freed inside the call; all are
 * synchronous.
 * ------------------------------------------------------------------------ */

/* Y[:, c] = A X[:, c] for c < ncols, A = Kx or Mx of `space` (matrix-free
 * stencil SpMM; Sec. 3 spatial matrices).  X: Nh x ncols (ldx), Y: Nh x ncols
 * (ldy); X and Y must not overlap.  ncols <= 16. */
sts_status sts_apply_op(const sts_space* space, int32_t op, const double* X, int64_t ldx,
                        double* Y, int64_t ldy, int32_t ncols, void* stream);

/* Conjugate gradients on A X[:, c] = B[:, c] with A = Kx or Mx per column
 * (ops[c]), X0 = 0, stopping when ||r|| <= rtol ||b|| or after maxit
 * iterations.  iters (host, length ncols, may be NULL) receives the
 * iteration count of each column.  ncols <= 8.  Returns STS_E_NUMERIC on a
 * non-positive curvature and STS_E_NOT_CONVERGED if a column hits maxit. */
sts_status sts_cg(const sts_space* space, const int32_t* ops, const double* B, int64_t ldb,
                  double* X, int64_t ldx, int32_t ncols, double rtol, int32_t maxit,
                  int32_t* iters, void* stream);

/* Kx X[:, c] = B[:, c] for c < ncols by conjugate gradients preconditioned
 * with one geometric multigrid V-cycle (the inner Kx^{-1} applications of
 * the extended Krylov space, Sec. 4; the preconditioner is this library's
 * choice, not the paper's).  X0 = 0; stops when ||r|| <= rtol ||b|| or after
 * maxit iterations.  Spaces (else STS_E_INVALID):
 *  - STS_FE_P1_2D with n <= 63, or n odd halving, n -> (n-1)/2 (odd at every
 *    step), at least once and down to at most 255 (e.g. 1023, 511, 255, 127,
 *    95);
 *  - STS_FE_Q1_3D_7PT (seven-point stiffness) with n <= 63 (the V-cycle is then
 *    the exact solve), or n odd halving down to at most 63 (e.g. 511, 255,
 *    127, 95).
 * B: Nh x ncols (ldb), X: Nh x ncols (ldx), device.  iters (host, may be
 * NULL) as for sts_cg.  ncols <= 8.  Same errors as sts_cg. */
sts_status sts_pcg_mg(const sts_space* space, const double* B, int64_t ldb, double* X,
                      int64_t ldx, int32_t ncols, double rtol, int32_t maxit, int32_t* iters,
                      void* stream);

/* Mx X[:, c] = B[:, c] for c < ncols (the Mx^{-1} applications of the
 * extended Krylov space, Sec. 4; the solvers are this library's choice).
 * 2-D P1: Chebyshev iteration -- the spectrum of diag(Mx)^{-1} Mx lies in
 * [1/2, 2], so k steps guarantee ||r|| <= 2 (1/3)^k ||b||; k is the smallest
 * count meeting rtol (at most 64) and is written to iters (host, may be NULL).
 * 3-D trilinear (cubic grids): Mx = (h/6)^3 T (x) T (x) T, T = tridiag(1, 4, 1),
 * solved directly by three passes of tridiagonal solves along the grid lines
 * (iters = 1).  Other spaces: STS_E_INVALID.  B, X: Nh x ncols (ldb, ldx),
 * device, ncols <= 8; for the 3-D solve X may equal B. */
sts_status sts_mass_solve(const sts_space* space, const double* B, int64_t ldb, double* X,
                          int64_t ldx, int32_t ncols, double rtol, int32_t* iters,
                          void* stream);

/* The preconditioner of sts_pcg_mg: Z[:, c] = Bmg R[:, c], one V-cycle from
 * zero: Chebyshev smoothing before and after each coarse correction (2-D:
 * three steps for the interval [1/2, 2] of the spectrum of diag(Kx)^{-1} Kx;
 * 3-D: two steps for [1/3, 2]); P1 interpolation and its transpose between
 * the nested meshes (3-D: of the Kuhn triangulation, whose P1 stiffness is
 * the seven-point stencil); the coarsest level solved exactly by the discrete
 * sine transform.  Bmg is symmetric positive definite.
 * Same spaces as sts_pcg_mg.  R: Nh x ncols (ldr), Z: Nh x ncols (ldz),
 * device, ncols <= 8. */
sts_status sts_mg_vcycle(const sts_space* space, const double* R, int64_t ldr, double* Z,
                         int64_t ldz, int32_t ncols, void* stream);

/* The V-cycle for Kx + shift Mx (shift >= 0), the preconditioner of the
 * shifted solves of the rational Krylov space (Sec. 4).  Every level's
 * operator is the coarse Kx + shift Mx, smoothed as in sts_mg_vcycle with its
 * own diagonal.
 *  - 2-D P1: P^T Mx P is the coarse mass for nested P1 spaces; the coarsest
 *    sine-transform solve takes the mass without its SW-NE coupling,
 *    (h^2/12)(6; 1 x 4), which the transform diagonalises.
 *  - 3-D: the coarse levels rediscretise the Q1 mass (it is not a Galerkin
 *    product of the Kuhn-mesh interpolation); the coarsest solve is exact,
 *    since tridiag(1, 4, 1) has the sine eigenvectors too.
 * Symmetric positive definite.  Same spaces, layout and errors as
 * sts_mg_vcycle; STS_E_INVALID for a negative shift. */
sts_status sts_mg_vcycle_shifted(const sts_space* space, double shift, const double* R,
                                 int64_t ldr, double* Z, int64_t ldz, int32_t ncols,
                                 void* stream);

/* Mixed precision (the FP32 bulk / FP64 accuracy split of the solves):
 * sts_mg_vcycle_shifted with the V-cycle's vectors stored in FP32 -- the
 * pre-smoothed iterates, residuals and Chebyshev directions of the finest
 * level and every vector of the coarser ones, the exact coarsest solve
 * included; R and Z stay FP64 and every operation is computed in FP64, so Z
 * differs from the FP64 V-cycle's by rounding to single precision (relative
 * about 1e-7), not by a different operator.  The V-cycle's bytes per node fall
 * by about a third.  Spaces: 3-D seven-point with n > 63 halving to <= 63
 * (STS_E_INVALID otherwise, and for a negative shift).  Layout as
 * sts_mg_vcycle. */
sts_status sts_mg_vcycle_mixed(const sts_space* space, double shift, const double* R, int64_t ldr,
                               double* Z, int64_t ldz, int32_t ncols, void* stream);

/* (Kx + shift Mx) X[:, c] = B[:, c] by FP64 conjugate gradients preconditioned
 * with sts_mg_vcycle_mixed.  The FP32 rounding perturbs the preconditioner, not
 * the operator or the residual recurrence, so the iteration reaches rtol as the
 * FP64 one does (the CG iteration acts as the FP64 refinement of the FP32
 * preconditioner).  Same spaces as sts_mg_vcycle_mixed; arguments, iters and
 * errors as sts_pcg_mg. */
sts_status sts_pcg_mg_mixed(const sts_space* space, double shift, const double* B, int64_t ldb,
                            double* X, int64_t ldx, int32_t ncols, double rtol, int32_t maxit,
                            int32_t* iters, void* stream);

/* Kx X = B for the 3-D seven-point stiffness with FP32 bulk work: FP32
 * multigrid PCG (vectors, stencil product, V-cycle and per-tile inner
 * products in FP32) as the correction solver of FP64 iterative refinement
 * (x += d, r = B - Kx x in FP64, until ||r|| <= rtol ||b|| per column; FP64
 * PCG finishes a column whose FP32 rounds stall).  These are the Kx solves
 * of the extended Krylov expansion (Sec. 4, the pole 0) under
 * sts_opts.mixed.  Needs a grid with a smoothed level (n > 63, halving to
 * <= 63).  B, X device, Nh x ncols (ldb, ldx >= Nh), 1 <= ncols <= 8;
 * 0 < rtol < 1.  *iters_fp32 / *iters_fp64 (nullable) receive the FP32 and
 * FP64 PCG iterations over all columns, *rounds the defect corrections.
 * Synchronous.  Errors: STS_E_INVALID; STS_E_NUMERIC for a non-finite
 * residual or a breakdown of the FP64 finish. */
sts_status sts_pcg_mg_refined(const sts_space* space, const double* B, int64_t ldb, double* X,
                              int64_t ldx, int32_t ncols, double rtol, int32_t maxit,
                              int64_t* iters_fp32, int64_t* iters_fp64, int64_t* rounds,
                              void* stream);

/* Direct solves A X[:, c] = B[:, c], A = Kx or Mx per column (ops[c]), for a
 * 1-D P1 space (STS_FE_P1_1D; else STS_E_INVALID): both matrices of Sec. 3
 * are constant-coefficient symmetric tridiagonal, solved by elimination
 * without pivoting (the inner solves of the extended Krylov space, Sec. 4)
 * in a nested-dissection order: 63-row blocks in parallel, the separators'
 * Schur complement recursively in LDS (up to 262208 nodes; longer grids
 * take one sequential sweep per column).  B, X: Nh x ncols (ldb, ldx >= Nh),
 * device, must not overlap; 1 <= ncols <= 8.  Synchronous. */
sts_status sts_tridiag_solve(const sts_space* space, const int32_t* ops, const double* B,
                             int64_t ldb, double* X, int64_t ldx, int32_t ncols, void* stream);

/* The adaptive shift rule of the rational Krylov space (Sec. 4 leaves the
 * rule to the literature it cites; this is the greedy choice of Druskin and
 * Simoncini for real spectra): the maximiser, over `grid` logarithmically
 * spaced points of [a, b] (end points included), of
 *     prod_l |s - shifts[l]| / prod_i |s + ritz[i]|,
 * evaluated in logarithms.  Host arrays; *s receives the shift.  Errors:
 * STS_E_INVALID unless 0 < a <= b and grid >= 2. */
sts_status sts_adaptive_shift(const double* ritz, int32_t k, const double* shifts, int32_t m,
                              double a, double b, int32_t grid, double* s);

/* (Kx + shift Mx) X[:, c] = B[:, c] (shift >= 0) as the rational Krylov steps
 * solve them: 1-D P1 spaces directly (elimination); 2-D and 3-D spaces that
 * the multigrid accepts by CG preconditioned with sts_mg_vcycle_shifted;
 * other spaces by CG; the iterations stop at relative residual rtol (at most
 * maxit; iters as for sts_cg).  B, X: Nh x ncols (ldb, ldx), device;
 * ncols <= 8. */
sts_status sts_shifted_solve(const sts_space* space, double shift, const double* B, int64_t ldb,
                             double* X, int64_t ldx, int32_t ncols, double rtol, int32_t maxit,
                             int32_t* iters, void* stream);

/* Block Gram-Schmidt in the Mx inner product: orthogonalise the ncols columns
 * of W (in place, Nh x ncols, ldw) against V (Nh x k, Mx-orthonormal, with
 * MV = Mx V given) twice (CGS2), then orthonormalise them by two Cholesky-QR
 * passes, dropping columns whose Mx-norm fell below defl_tol of their norm on
 * entry.  The kept, orthonormal columns are packed to the front of W, and
 * MW (Nh x ncols, ldw) receives Mx times them.  *kept (host) is the number of
 * kept columns and keep_idx (host, length ncols, may be NULL) their original
 * indices.  ncols <= 8. */
sts_status sts_m_orthonormalize(const sts_space* space, const double* V, const double* MV,
                                int64_t ldv, int64_t k, double* W, double* MW, int64_t ldw,
                                int32_t ncols, double defl_tol, int32_t* kept,
                                int32_t* keep_idx, void* stream);

/* The contraction of block Gram-Schmidt, C (m x n, ldc) = A^T B, for a tall
 * A (rows x m, lda) and a thin B (rows x n, ldb), n <= 16; FP64 matrix cores.
 * With A = Mx V it gives the coefficients that orthogonalise a new block
 * against the basis, whose columns Sec. 4 takes orthonormal.  All pointers
 * device; rows >= 0, m >= 1, 1 <= n <= 16, ldc >= m; A and B must not overlap
 * C; scratch is allocated and freed inside the call.  Errors: STS_E_INVALID
 * for sizes out of range or ld < rows. */
sts_status sts_gram(int64_t rows, int32_t m, int32_t n, const double* A, int64_t lda,
                    const double* B, int64_t ldb, double* C, int64_t ldc, void* stream);

/* sts_gram for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, hosts that forbid hipMalloc): the same
 * contraction C (m x n, ldc) = A^T B with the same kernels, its partial
 * products kept in a device array built into the library (16 MiB, one copy
 * per device, held until the process ends) instead of memory allocated per
 * call.  Calls no hipMalloc / hipFree.  Asynchronous: the work is ordered on
 * `stream` and C is ready when the stream reaches it.  Every call on a device
 * uses that device's one array, so calls that overlap on a device (other
 * streams, other host threads) race; nothing needs clearing between calls.
 * Sizes and pointers as for sts_gram, and m <= 512.  Errors: STS_E_INVALID
 * for sizes out of range (m > 512 included), STS_E_DEVICE if the array's
 * device address cannot be obtained or a launch fails. */
sts_status sts_gram_noalloc(int64_t rows, int32_t m, int32_t n, const double* A, int64_t lda,
                            const double* B, int64_t ldb, double* C, int64_t ldc, void* stream);

/* The basis update of block Gram-Schmidt, W (rows x n, ldw) -= A (rows x m,
 * lda) C (m x n, ldc), n <= 16; FP64 matrix cores.  With A = V and C from
 * sts_gram it removes the new block's components along the orthonormal basis
 * of Sec. 4.  All pointers device; W must not overlap A or C.  Errors:
 * STS_E_INVALID for n > 16 or ld < rows. */
sts_status sts_basis_update(int64_t rows, int32_t m, int32_t n, const double* A, int64_t lda,
                            const double* C, int64_t ldc, double* W, int64_t ldw, void* stream);

/* The contraction of sts_gram in FP32, as the first Gram-Schmidt pass of the
 * mixed-precision solve (sts_opts.mixed) runs it against the FP32 copy of the
 * basis for its coefficients: C (m x n, FP64 storage) = A^T B with A FP32
 * (rows x m, lda) and B FP64 rounded to FP32 as it is read.  Products and
 * sums are FP32 on the matrix cores (relative accuracy about 1e-7 of
 * |A|^T |B|).  The solve removes these coefficients with the FP64 basis and
 * re-orthogonalises in FP64, keeping the Mx-orthonormal basis of Sec. 4 in
 * the span of the expansion.  Sizes, pointers and errors as for sts_gram;
 * synchronous. */
sts_status sts_gram_fp32(int64_t rows, int32_t m, int32_t n, const float* A, int64_t lda,
                         const double* B, int64_t ldb, double* C, int64_t ldc, void* stream);

/* Eigendecomposition of a symmetric k x k matrix A (lda): A Q = Q diag(lam),
 * Q^T Q = I, by Householder tridiagonalisation, bisection, inverse iteration
 * and Newton-Schulz orthogonalisation.  lam: k,
 * Q: k x k (ldq).  For the reduced pencil (Km, Mm) of an Mx-orthonormal basis
 * Mm = I up to rounding, so this diagonalises the pencil (Sec. 4, reduced
 * equation). */
sts_status sts_sym_eig(int64_t k, const double* A, int64_t lda, double* lam, double* Q,
                       int64_t ldq, void* stream);

/* Reduced time sweep: Y = Q Z where each row z_i solves the lower-bidiagonal
 * recurrence (Dt + lam_i Mt) z_i = (Q^T beta F2^T)[i, :] (Sec. 4 reduced
 * equation after diagonalising the spatial pencil).  lam: k, Q: k x k (ldq),
 * beta: k x p (ldb), F2: nt x p (ldf), Dt/Mt host bidiagonals, Y: k x nt (ldy). */
sts_status sts_time_sweep(int64_t k, int64_t nt, int32_t p, const double* lam, const double* Q,
                          int64_t ldq, const double* beta, int64_t ldb, const double* F2,
                          int64_t ldf, const sts_bidiag* Dt, const sts_bidiag* Mt, double* Y,
                          int64_t ldy, void* stream);

/* ------------------------------------------------------------------------
 * Many independent problems on one GPU.
 *
 * Each problem of a batch is the method of Sec. 4 applied to its own data;
 * the pool only schedules whole solves.  A pool owns `workers` host threads'
 * worth of HIP streams (non-blocking, default priority) on the device that
 * is current at creation.  sts_pool_solve runs sts_solve on every problem,
 * up to `workers` at a time, taking the problems in order of decreasing
 * estimated cost (grid size, columns, time steps).  While a problem is being
 * solved it is bound to its worker's stream; before and after, the work on
 * its own stream is waited for, so the caller may queue work on that stream
 * before the call and use the factors after it.  Factors are bitwise those of
 * solving each problem alone.
 * ------------------------------------------------------------------------ */
typedef struct sts_pool sts_pool;

/* workers: 1..64.  Errors: STS_E_INVALID, STS_E_DEVICE (stream creation). */
sts_status sts_pool_create(int32_t workers, sts_pool** out);

/* Number of workers of the pool. */
sts_status sts_pool_workers(const sts_pool* pool, int32_t* workers);

/* Solve probs[0..n).  opts: nopts = 0 (defaults for all), 1 (opts[0] for all)
 * or n (opts[i] for problem i).  infos (n entries) and status (n entries)
 * may be NULL.  A problem may appear only once; problems must not be used by
 * other threads during the call.  Returns STS_OK if every solve returned
 * STS_OK, else the status of the lowest-index failing problem (the others
 * still run to completion; status[] holds each one's result, and
 * sts_last_error names the failing problem).  Synchronous. */
sts_status sts_pool_solve(sts_pool* pool, int32_t n, sts_problem* const* probs,
                          const sts_opts* opts, int32_t nopts, sts_info* infos,
                          sts_status* status);

/* Destroy the pool (NULL-safe).  Must not overlap an sts_pool_solve. */
void sts_pool_destroy(sts_pool* pool);

/* ------------------------------------------------------------------------
 * Serving: a request queue in front of the solver.
 *
 * A request is one problem of Sec. 2-4 (space, time matrices, low-rank load,
 * options).  sts_server_submit copies its host inputs and returns a ticket at
 * once.  `workers` worker threads, each with its own non-blocking HIP stream
 * on the device current at creation, take requests first come, first served.
 * A request is admitted only when its device-memory footprint (sts_footprint)
 * fits in mem_budget next to the requests admitted and not yet released; a
 * request that could never fit is refused at submission (STS_E_NOMEM).  A
 * finished request keeps its problem (basis and factors) in device memory
 * until sts_server_release.  Factors are bitwise those of the same request
 * solved alone.
 * ------------------------------------------------------------------------ */
typedef struct sts_server sts_server;

typedef struct {
  sts_space space;
  int64_t nt;               /* time steps */
  int32_t p;                /* rank of the load, 1..4 */
  int32_t pad_;
  const double* dt_diag;    /* host: Dt diagonal (nt) and sub-diagonal (nt-1) */
  const double* dt_sub;
  const double* mt_diag;    /* host: Mt diagonal (nt) and sub-diagonal (nt-1) */
  const double* mt_sub;
  const double* F1;         /* host: Nh x p, leading dimension ldf1 */
  int64_t ldf1;
  const double* F2;         /* host: nt x p, leading dimension ldf2 */
  int64_t ldf2;
  sts_opts opts;            /* solve options (start from sts_default_opts) */
} sts_request;

typedef struct {
  int32_t status;           /* sts_status of the request's create and solve */
  int32_t pad_;
  double queued_seconds;    /* submission -> admission */
  double latency_seconds;   /* submission -> factors ready in device memory */
  int64_t footprint;        /* device bytes reserved for the request */
  sts_info info;            /* of the solve */
} sts_result;

typedef struct {
  int64_t submitted, completed, released;
  int64_t queued, running;
  int64_t mem_in_use, mem_peak, mem_budget;   /* bytes of footprint */
} sts_server_stats;

/* Device bytes a problem of this shape holds after sts_create and the first
 * basis capacity a solve with these options (NULL = defaults) maps: inputs,
 * inner-solve work and 3 Nh doubles for each of min(8, max_outer + 2) blocks
 * of 2p columns.  The basis then grows by 3 Nh doubles per column as the
 * space grows (sts_solve).  -1 for an invalid shape. */
int64_t sts_footprint(const sts_space* space, int64_t nt, int32_t p, const sts_opts* opts);

/* workers: 1..64; mem_budget > 0 bytes.  Errors: STS_E_INVALID, STS_E_DEVICE. */
sts_status sts_server_create(int32_t workers, int64_t mem_budget, sts_server** out);

/* Queue a request; *ticket identifies it.  The inputs are copied before the
 * call returns.  Errors: STS_E_INVALID (shape, pointers, leading dimensions;
 * the full validation of sts_create happens when the request runs and is
 * reported in its sts_result), STS_E_NOMEM (footprint above the budget),
 * STS_E_STATE (server shutting down). */
sts_status sts_server_submit(sts_server* server, const sts_request* req, int64_t* ticket);

/* Wait up to timeout_s seconds (< 0: without limit) for the request to
 * finish; then fill *result (may be NULL) and *prob (may be NULL) with the
 * solved problem, which the server owns until sts_server_release (use it
 * with sts_get_factors, sts_true_residual, ...; do not destroy it).
 * STS_E_STATE if the request has not finished in time, STS_E_INVALID for an
 * unknown or released ticket.  A failed request returns STS_OK here with its
 * status in result->status (sts_last_error describes it). */
sts_status sts_server_wait(sts_server* server, int64_t ticket, double timeout_s,
                           sts_result* result, sts_problem** prob);

/* Free a finished request's problem and its footprint.  STS_E_STATE if it
 * has not finished. */
sts_status sts_server_release(sts_server* server, int64_t ticket);

sts_status sts_server_get_stats(sts_server* server, sts_server_stats* out);

/* Stop the workers after their current requests, drop queued requests and
 * free every unreleased problem (NULL-safe).  No other call may overlap. */
void sts_server_destroy(sts_server* server);

#ifdef __cplusplus
}
#endif

#endif /* STS_H */
