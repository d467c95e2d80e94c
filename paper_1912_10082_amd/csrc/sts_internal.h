// Internal declarations shared by the HIP kernels and the host driver.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/sts.h"

namespace sts {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

void set_error(const std::string& msg);

struct Error {
  sts_status code;
  std::string msg;
};

#define STS_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::sts::Error{STS_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define STS_REQUIRE(cond, code, msg)                      \
  do {                                                    \
    if (!(cond)) throw ::sts::Error{(code), (msg)};       \
  } while (0)

// ---------------------------------------------------------------------------
// kernel profiling (opts.profile = 1)
// ---------------------------------------------------------------------------

// Per-launch start/stop events attached to the dispatches themselves
// (hipExtLaunchKernel), with the algorithmic bytes of each launch; the
// elapsed times are read only when asked for, after the timed work.
struct Profiler {
  std::vector<hipEvent_t> pool;   // start / stop pairs
  std::vector<int> ids;
  std::vector<double> bytes;
  double sec[STS_K_COUNT] = {};
  int64_t cnt[STS_K_COUNT] = {};
  double byt[STS_K_COUNT] = {};
  bool collected = false;
  Profiler() = default;
  Profiler(const Profiler&) = delete;
  Profiler& operator=(const Profiler&) = delete;
  ~Profiler();
  void reset();
  void next(int kid, double b, hipEvent_t* s, hipEvent_t* e);
  void collect();
};
// The profiler of the calling thread's current solve, or null.
Profiler* active_profiler();
void set_active_profiler(Profiler* p);

template <std::size_t... I, typename Tup>
inline void arg_ptrs(Tup& t, void** out, std::index_sequence<I...>) {
  ((out[I] = static_cast<void*>(&std::get<I>(t))), ...);
}

// Launch a kernel; under an active profiler with start/stop events.
template <typename... KArgs, typename... Args>
inline void launch(int kid, double bytes, void (*kernel)(KArgs...), dim3 grid, dim3 block,
                   unsigned shmem, hipStream_t st, Args&&... args) {
  static_assert(sizeof...(KArgs) == sizeof...(Args), "kernel argument count");
  std::tuple<KArgs...> tup(std::forward<Args>(args)...);
  void* ptrs[sizeof...(KArgs) > 0 ? sizeof...(KArgs) : 1];
  arg_ptrs(tup, ptrs, std::index_sequence_for<KArgs...>{});
  hipEvent_t s = nullptr, e = nullptr;
  if (Profiler* p = active_profiler()) p->next(kid, bytes, &s, &e);
  hipError_t err = hipExtLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, ptrs,
                                      shmem, st, s, e, 0);
  if (err != hipSuccess)
    throw Error{STS_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(err)};
}

// ---------------------------------------------------------------------------
// spatial operators as constant-coefficient stencils
// ---------------------------------------------------------------------------

// A constant-coefficient stencil on an nx x ny x nz box of interior nodes
// (x fastest) with zero Dirichlet values outside.  c[(dz+1)*9 + (dy+1)*3 +
// (dx+1)] multiplies the neighbour at offset (dx, dy, dz).
struct Stencil {
  int dim;
  int nx, ny, nz;
  double c[27];
};

struct Grid {
  int dim;
  int nx, ny, nz;
  int64_t nh;
};

// Kx (op = STS_OP_K) or Mx (STS_OP_M) of a space descriptor (validated).
Stencil make_stencil(const sts_space& s, int op);
Grid make_grid(const sts_space& s);
void validate_space(const sts_space* s);

// ---------------------------------------------------------------------------
// CG state shared by host and device
// ---------------------------------------------------------------------------

constexpr int kMaxCols = 8;     // columns in one CG batch (2P, P <= 4)

// Per-column CG state.  Iteration i of a column uses gamma_i = (r_i, r_i) and
// delta_i = (A r_i, r_i) of the residual entering it, plus alpha_{i-1} and
// gamma_{i-1} kept here; `iters` counts completed iterations.
struct CGScal {
  double alpha;   // alpha of the last completed iteration
  double gamma;   // gamma of the residual that entered it
  double gamma0;  // (b, b)
  double rtol2;   // stop when gamma_i <= rtol2 * gamma0
  int active;     // 1 while the column iterates
  int iters;      // completed iterations
  int maxit;
  int flag;       // 0 running, 1 converged, 2 hit maxit, 3 breakdown / non-finite
  double rho;     // preconditioned CG: (r, z) of the current direction
};

// The state and the per-tile partial sums are double-buffered by launch
// parity: launch k reads slot (k-1) & 1 and writes slot k & 1.
struct CGWork {
  // device buffers, column-major nh x ncols with leading dimension ld; r and
  // p are pairs (launch k reads buffer (k-1) & 1, writes buffer k & 1)
  double* x;
  double* r[2];
  double* p[2];
  int64_t ld;
  CGScal* scal;         // device, 2 * kMaxCols entries (two slots)
  double* partials;     // device, 2 slots * kMaxCols * max_tiles * 2
  int max_tiles;
  const double* b[kMaxCols];   // right-hand-side columns (set-up only)
};

// Initial state of a CG batch (both slots): columns c < ncols active.
void cg_init_state(const CGWork& w, int ncols, double rtol, int maxit, hipStream_t st);
// Set-up: r = b, p = 0, x = 0, partials of (b, b) and (A b, b) into slot 0.
// cg_init_state has written the initial state.
void cg_setup(const Grid& g, const Stencil& K, const Stencil& M, const int* ops, int ncols,
              const CGWork& w, hipStream_t st);
// One CG iteration; `parity` = launch index & 1 (the set-up is launch 0).
// Work-groups are launched for the columns in cols[0..nlaunch) (the host's
// possibly stale view of the active ones); every launch updates the state of
// all ncols columns, and a launched column that has stopped costs one tile
// load per work-group.
void cg_iterate(const Grid& g, const Stencil& K, const Stencil& M, const int* ops, int ncols,
                const CGWork& w, int parity, const int* cols, int nlaunch, hipStream_t st);
int cg_tiles(const Grid& g);

// Y[:, c] = A_c X[:, c], A_c = ops[c] ? M : K (ncols <= 16)
void stencil_apply(const Grid& g, const Stencil& K, const Stencil& M, const int* ops, int ncols,
                   const double* X, int64_t ldx, double* Y, int64_t ldy, hipStream_t st);
// KX = Kx X and MX = Mx X (ncols <= 16 columns) from one read of X.
void stencil_apply_km(const Grid& g, const Stencil& K, const Stencil& M, int ncols,
                      const double* X, int64_t ldx, double* KX, int64_t ldk, double* MX,
                      int64_t ldm, hipStream_t st);

// ---------------------------------------------------------------------------
// multigrid-preconditioned CG for the 2-D P1 and 3-D seven-point stiffness
// ---------------------------------------------------------------------------

constexpr int kMGMaxLevels = 12;
constexpr int kMGCoarseMax = 63;   // coarsest levels up to this size: one work-group per column
constexpr int kMGExactMax = 255;   // largest exactly solved (coarsest) level
constexpr int kMGNu = 3;           // Chebyshev smoothing steps before and after
constexpr int kMG3ExactMax = 63;   // 3-D: largest exactly solved (coarsest) level

struct MGPlan {
  int dim;                   // 2: five-point P1 stiffness, 3: seven-point stiffness
  int nlev;                  // smoothed levels 0..nlev-1; level nlev is solved exactly
  int n[kMGMaxLevels + 1];   // nodes per direction, n[l+1] = (n[l] - 1) / 2
  int exact;                 // size of the exactly solved coarsest level (= n[nlev])
  double mu;                 // 2-D: Kx = mu (4; -1 x 4) on every level;
                             // 3-D: Kx = mu (6; -1 x 6) on level 0, 2^l mu on level l
  double sw0;                // Kx + s Mx: s times the level-0 mass scale (2-D h^2 / 12,
                             // 3-D (h/6)^3); 0: Kx alone
  int f32;                   // 3-D with nlev >= 1: the V-cycle stores its vectors in FP32
                             // (all but the finest right-hand side and result)
  int f32cg;                 // 3-D with nlev >= 1: FP32 PCG -- x, r, z, p, q and every
                             // V-cycle vector in FP32, FP32 vector arithmetic in the PCG
  int x64;                   // with f32cg: x accumulated in FP64 (x += alpha p), so that
                             // the residual can be replaced by b - K x (mg3_replace)
};
// The m x m sine-transform matrix (row-major) followed by the m eigenvalues
// 2 - 2 cos(pi j / (m + 1)) of tridiag(-1, 2, -1): m (m + 1) doubles.
void mg_dst_table(int m, double* out);
size_t mg_dst_table_size(int m);   // doubles written by mg_dst_table
// True (and *plan filled) if Kx is the 2-D five-point P1 stiffness on a square
// grid that halves, n -> (n-1)/2, down to at most kMGExactMax nodes, or the
// 3-D seven-point stiffness on a cube that halves down to kMG3ExactMax.
bool mg_plan(const Grid& g, const Stencil& K, MGPlan* plan);
bool mg3_plan(const Grid& g, const Stencil& K, MGPlan* plan);
int mg3_max_tiles(const MGPlan& p);
// Algorithmic bytes of one 3-D column-iteration per fine node.
double mg3_bytes_per_node(const MGPlan& p);
// Partial-sum slots per column the PCG kernels need.
int mg_max_tiles(const MGPlan& p);

struct MGWork {
  MGPlan plan;
  double* b[kMGMaxLevels + 1];   // right-hand side per level; b[0] is the PCG residual r
  double* e[kMGMaxLevels + 1];   // V-cycle result per level; e[0] is z
  double* xp[kMGMaxLevels + 1];  // pre-smoothed iterate per smoothed level (stride ld)
  double* u1[kMGMaxLevels + 1];  // 3-D: iterate after the first post-smoothing step
  double* d0[kMGMaxLevels + 1];  // 3-D: its Chebyshev direction
  int64_t ld[kMGMaxLevels + 1];  // column stride per level
  double* x;                     // solution columns (x + c * ldx)
  int64_t ldx;
  double* p[2];                  // search directions (stride ld[0]), by parity
  double* q;                     // K p
  CGScal* scal;                  // 2 slots of kMaxCols
  double* part_rr;               // kMaxCols * max_tiles each
  double* part_rz;
  double* part_pq;
  double* alpha;                 // kMaxCols
  double* tot;                   // 3 x kMaxCols: summed partials (3-D, large grids)
  int max_tiles;
  const double* dst;             // device copy of mg_dst_table(plan.exact)
  double* t1;                    // coarsest-level temporaries above kMGCoarseMax
  double* t2;                    //   (stride ld[nlev], kMaxCols columns)
  const double* col_rtol;        // host, per column (set-up), or null: the scalar rtol
  const double* rhs[kMaxCols];   // right-hand side of each column of the current run
};
// e[0][:, c] = B b[0][:, c] (one V-cycle) for the columns cols[0..nlaunch);
// columns whose state in `act` (may be null) is inactive are skipped; with
// `partials` the per-tile (b, e) sums go to part_rz.
void mg_vcycle(const MGWork& w, const CGScal* act, const int* cols, int nlaunch, bool partials,
               hipStream_t st);
// PCG set-up for K x_c = b[j] (c = cols[j]): x = 0, r = b, state slots of
// columns c < ncols (active if launched).
void pcg_setup(const MGWork& w, const double* const* b, const int* cols, int nlaunch, int ncols,
               double rtol, int maxit, hipStream_t st);
// One PCG iteration (V-cycle, A, B) writing state slot `parity`.
void pcg_iterate(const MGWork& w, int parity, const int* cols, int nlaunch, int ncols,
                 hipStream_t st);
// The 3-D forms of the three calls above (mg_vcycle, pcg_setup and
// pcg_iterate dispatch on plan.dim).
void mg3_vcycle(const MGWork& w, const CGScal* act, const int* cols, int nlaunch, bool partials,
                hipStream_t st);
void pcg3_setup(const MGWork& w, const double* const* b, const int* cols, int nlaunch, int ncols,
                double rtol, int maxit, hipStream_t st);
void pcg3_iterate(const MGWork& w, int parity, const int* cols, int nlaunch, int ncols,
                  hipStream_t st);
// Defect correction of the 3-D FP32 inner solves, in FP64: for slot j <
// ncols, x[j] += d[j] (FP32 if d32, else FP64; d or d[j] null: x[j]
// unchanged), r[j] = b[j] - (Kx + s Mx) x[j] and norms2[j] = (r[j], r[j])
// (device).  Every vector is one fine-grid column.  Uses w.part_rr.
void mg3_defect(const MGWork& w, int ncols, double* const* x, const void* const* d, bool d32,
                const double* const* b, double* const* r, double* norms2, hipStream_t st);
// Residual replacement in the FP32 PCG with x in FP64 (plan.f32cg, plan.x64):
// for the columns cols[0..nl), r = rhs - (Kx + s Mx) x in FP64, stored to the
// PCG's FP32 residual, with its FP64 per-tile (r, r) partials in part_rr.
void mg3_replace(const MGWork& w, const int* cols, int nl, hipStream_t st);

// ---------------------------------------------------------------------------
// Mx solves by Chebyshev iteration (2-D P1 mass matrix)
// ---------------------------------------------------------------------------

constexpr int kMassSteps = 6;       // Chebyshev steps fused per launch (= LDS halo)
constexpr int kMassMaxIters = 64;

// Steps for ||r|| <= rtol ||b|| (the bound 2 (1/3)^k).
int mass_cheb_iters(double rtol);
// True if Mx is the 2-D P1 mass stencil w (6; 1 at E, W, N, S, NE, SW).
bool mass_cheb_supported(const Grid& g, const Stencil& M);
// x[:, c] = Mx^{-1} b[c] for c < ncols after `iters` steps; xbuf / dbuf: two
// state buffers each (stride ld, kMaxCols columns).
void mass_cheb_solve(const Grid& g, const Stencil& M, int ncols, const double* const* b,
                     double* x, int64_t ldx, double* xbuf[2], double* dbuf[2], int64_t ld,
                     int iters, hipStream_t st);

// ---------------------------------------------------------------------------
// dense tall-skinny kernels (FP64 MFMA)
// ---------------------------------------------------------------------------

// C (m x n, ldc) = A^T B with A: rows x m (lda), B: rows x n (ldb), n <= 16.
// partial: device scratch of gemm_tn_partial_size(rows, m) doubles.
void gemm_tn(int64_t rows, int m, int n, const double* A, int64_t lda, const double* B,
             int64_t ldb, double* C, int64_t ldc, double* partial, hipStream_t st);
int64_t gemm_tn_partial_size(int64_t rows, int m);

// C_s (m x nb[s], ldc[s]) = A^T B_s for up to three column segments B_s (rows
// x nb[s], common ldb), 32 columns in all, in one pass over A (partial:
// gemm_tn_partial_size_wide(rows, m) doubles).
int64_t gemm_tn_partial_size_wide(int64_t rows, int m);
void gemm_tn_segs(int64_t rows, int m, const double* A, int64_t lda, int nseg,
                  const double* const* B, const int* nb, int64_t ldb, double* const* C,
                  const int64_t* ldc, double* partial, hipStream_t st);

// [C1 C2] = A^T [B1 B2]: B1 rows x n1, B2 rows x n2 (common ldb), n1 + n2 <= 16;
// C1 (m x n1) and C2 (m x n2) share ldc.  One pass over A.
void gemm_tn2(int64_t rows, int m, int n1, int n2, const double* A, int64_t lda,
              const double* B1, const double* B2, int64_t ldb, double* C1, double* C2,
              int64_t ldc, double* partial, hipStream_t st);

// W (rows x n, ldw) -= A (rows x m, lda) C (m x n, ldc), n <= 16.
void gemm_nn_sub(int64_t rows, int m, int n, const double* A, int64_t lda, const double* C,
                 int64_t ldc, double* W, int64_t ldw, hipStream_t st);

// FP32 form for the coefficients of the first Gram-Schmidt pass of the
// mixed-precision solve: C (m x n, FP64 storage) = A^T B with A FP32 and B
// FP64 rounded to FP32, products and sums in FP32 (partial:
// gemm_tn_partial_size(rows, m) floats or more).
void gemm_tn32(int64_t rows, int m, int n, const float* A, int64_t lda, const double* B,
               int64_t ldb, double* C, int64_t ldc, float* partial, hipStream_t st);
// dst (FP32) = src (FP64) rounded, rows x ncols.
void round_cols(int64_t rows, int ncols, const double* src, int64_t lds, float* dst, int64_t ldd,
                hipStream_t st);

// D (m x n, ldd) = alpha op(A) B + beta D, op(A) = A (m x kk) or A^T (A kk x m);
// small/medium sizes.
void gemm_small(bool transA, int m, int n, int kk, double alpha, const double* A, int64_t lda,
                const double* B, int64_t ldb, double beta, double* D, int64_t ldd,
                hipStream_t st);

// D (m x n, ldd) = A (m x kk, lda) B (kk x n, ldb), small/medium sizes.
void gemm_nn(int m, int n, int kk, const double* A, int64_t lda, const double* B, int64_t ldb,
             double* D, int64_t ldd, hipStream_t st);

// ||[A_0 A_1 A_2] B||_F^2 without forming the product: A_s rows x m_s (lda_s),
// B (m_0+m_1+m_2) x n (ldb).  Result written to *out (device).
struct Seg {
  const double* A;
  int64_t lda;
  int m;
};
// upper: B[j][t] = 0 for j < t (B^T a triangular factor); those products are skipped.
void residual_norm2(int64_t rows, int n, const Seg* segs, int nseg, const double* B, int64_t ldb,
                    double* out, double* partial, unsigned* counter, hipStream_t st,
                    bool upper = false);
int64_t residual_norm2_partial_size(int64_t rows, int n);

// Upper-triangular factor of a rows x n matrix (rows >= n) by blocked
// Householder QR: A is overwritten, Rc (n x n, ld n) receives R with zeros
// below the diagonal.  work: qr_r_work_doubles(rows, n) doubles.
constexpr int kQrNb = 8;            // panel width
constexpr int kQrMaxRows = 4096;    // panel held in registers of 1024 threads
bool qr_r_supported(int64_t rows, int n);
size_t qr_r_work_doubles(int64_t rows, int n);
void qr_r(int64_t rows, int n, double* A, int64_t lda, double* Rc, double* work, hipStream_t st);

// ---------------------------------------------------------------------------
// small dense helpers (one work-group)
// ---------------------------------------------------------------------------

// Cholesky-QR step on the b x b Gram G (ldg) of a block: keeps, in order,
// the columns whose norm is at least defl_v times norm0[c] (skipped if norm0 is
// NULL) and whose part independent of the earlier kept columns is at least
// defl_b of their norm; writes R^{-1} of the kept block (upper triangular,
// b x b, ld b) and the kept count / indices to `info`.
struct CholInfo {
  int kept;
  int idx[16];
  int ok;
  double rmin;   // smallest independence ratio sqrt(d_j / G_jj) of a kept column
};
void chol_deflate(int b, const double* G, int64_t ldg, const double* norm0, double defl_v,
                  double defl_b, double* Rinv, CholInfo* info, hipStream_t st);
// Smallest block-internal independence the Gram-based test can resolve.
constexpr double kBlockDefl = 1e-7;

// Orthonormalise W (nh x ncols, ldw) against V (nh x k, Mx-orthonormal,
// MV = Mx V, ld ldv) and within itself in the Mx inner product: CGS2 against V,
// Cholesky-QR with deflation, one more CGS pass against V and a second
// Cholesky-QR.  Kept columns are packed to the front of W, MW = Mx W.
// Returns the kept count; idx[j] = source column of kept column j.
struct OrthScratch {
  double* part;   // gemm_tn partial, gemm_tn_partial_size(nh, max(k, 16))
  double* G;      // 256
  double* C;      // max(k, 1) * 16 (ld ldc)
  int64_t ldc;
  double* norm0;  // 16
  double* Rinv;   // 256
  CholInfo* info; // device
  CholInfo* host; // pinned host copy
  int cgs_passes; // out: FP64 Gram-Schmidt passes made against V (1 to 3)
  int cgs32_passes;       // out: FP32 passes (0 or 1)
  const float* V32 = nullptr;   // FP32 copy of V (same ld): the first pass in FP32
  // reduced-matrix columns of the previous block, formed in the second pass:
  // pend_Kout / pend_Mout (ld pend_ldc) = V^T pend_K / pend_M (pend_n columns)
  int pend_n = 0;
  const double* pend_K = nullptr;
  const double* pend_M = nullptr;
  double* pend_Kout = nullptr;
  double* pend_Mout = nullptr;
  int64_t pend_ldc = 0;
  bool pend_done = false;   // out: the pass formed them
};
int orthonormalize_block(const Grid& g, const Stencil& K, const Stencil& M, const double* V,
                         const double* MV, int64_t ldv, int64_t k, double* W, double* MW,
                         int64_t ldw, int ncols, double defl, OrthScratch& s, int* idx,
                         hipStream_t st, double* KW = nullptr, bool first_done = false);
// W[:, 0:kept] = W[:, idx] * Rinv (kept x kept upper triangular), also for MW.
void apply_rinv(int64_t rows, int b, const CholInfo* info, const double* Rinv, double* W,
                double* MW, int64_t ldw, double* tmp, hipStream_t st);

// ---------------------------------------------------------------------------
// reduced problem
// ---------------------------------------------------------------------------

constexpr int kEigMaxK = 2048;   // largest order of sym_eig
constexpr int kEigNB = 16;       // panel width of the tridiagonalisation

struct EigWork {
  double* base;   // eig_work_doubles(k) doubles of device scratch
  int* status;    // device: 0, or 1 if the input was not finite
};
int64_t eig_work_doubles(int k);
// Km Q = Q diag(lam) for a symmetric k x k matrix (ascending eigenvalues,
// orthonormal Q): Householder tridiagonalisation, multisection, inverse
// iteration, Rayleigh-Ritz correction, back-transformation.
void sym_eig(int k, const double* A, int64_t lda, double* lam, double* Q, int64_t ldq,
             const EigWork& w, hipStream_t st);
// Eigenvalues only (tridiagonalisation and bisection), ascending, into lam
// (device, k); same workspace as sym_eig.
void sym_eigvals(int k, const double* A, int64_t lda, double* lam, const EigWork& w,
                 hipStream_t st);

struct TimeOps {
  const double* d;   // Dt diagonal (nt)
  const double* e;   // Dt sub-diagonal (nt-1, e[l] = Dt[l+1, l])
  const double* m;   // Mt diagonal
  const double* n;   // Mt sub-diagonal
};
// Z (k x nt, ldz): (Dt + lam_i Mt) z_i = G_i with G = qb F2^T, qb = Q^T beta (k x p).
void time_sweep(int k, int nt, int p, const double* lam, const double* qb, int64_t ldqb,
                const double* F2, int64_t ldf, const TimeOps& t, double* Z, int64_t ldz,
                hipStream_t st);
// The same recurrences for a full right-hand side G (k x nt, ldg).
void time_sweep_full(int k, int nt, const double* lam, const double* G, int64_t ldg,
                     const TimeOps& t, double* Z, int64_t ldz, hipStream_t st);
// R (k x nt, ldr) = beta F2^T - KY Mt^T - Y Dt^T with KY = Km Y (both ldy):
// the residual of the reduced equation.
void reduced_residual(int k, int nt, int p, const double* beta, int64_t ldb, const double* F2,
                      int64_t ldf, const double* KY, const double* Y, int64_t ldy,
                      const TimeOps& t, double* R, int64_t ldr, hipStream_t st);
// out (nt x k, ldo) = scale * T A^T for A (k x nt) and a lower-bidiagonal T
// (diag td, sub ts): out[l, i] = scale (td[l] A[i, l] + ts[l-1] A[i, l-1]).
void bidiag_right(int k, int nt, const double* A, int64_t lda, const double* td, const double* ts,
                  double scale, double* out, int64_t ldo, hipStream_t st);
// ||L^T (T1 Mt^T)||_F^2 for T1 (b x nt), L (b x b lower, ldl); result to *out.
void cheap_residual(int b, int nt, const double* T1, int64_t ldt, const double* L, int64_t ldl,
                    const double* md, const double* ms, double* out, double* partial,
                    unsigned* counter, hipStream_t st);

// B (n x m, ldb) = A^T for A (m x n, lda).
void transpose(int m, int n, const double* A, int64_t lda, double* B, int64_t ldb, hipStream_t st);
// Lower Cholesky factor of a b x b SPD matrix (one thread); *ok = 0 if not SPD.
void chol_lower(int b, const double* G, int64_t ldg, double* L, int64_t ldl, int* ok,
                hipStream_t st);
// dst[c, r] = src[r, c] for the m x n block src (fills the mirror of a symmetric block).
void mirror(int m, int n, const double* src, int64_t lds, double* dst, int64_t ldd, hipStream_t st);

// Copy / fill helpers.
void copy_cols(int64_t rows, int ncols, const double* src, int64_t lds, double* dst, int64_t ldd,
               hipStream_t st);
void fill(double* p, int64_t n, double v, hipStream_t st);
// p[0..n) *= v (v = 0 stores zeros).
void scale(double* p, int64_t n, double v, hipStream_t st);
// sum of squares of a column-major block (deterministic), result to *out.
void sumsq(int64_t rows, int ncols, const double* A, int64_t lda, double* out, double* partial,
           unsigned* counter, hipStream_t st);

// ---------------------------------------------------------------------------
// direct tridiagonal inner solves (1-D P1), tridiag.hip
// ---------------------------------------------------------------------------
constexpr int kTriPeriod = 64;             // 63 block rows, then one separator row
constexpr int kTriMaxLevels = 8;
constexpr int64_t kTriMaxReduced = 4096;   // rows of the first reduced level held in LDS
// The levels of the blocked elimination of an Nh x Nh tridiagonal matrix:
// n[l] rows at level l (n[l + 1] = its separators), each level's seven factor
// arrays of ld[l] doubles at off[l]; total doubles per operator.  blocked is
// false where the first reduced level exceeds kTriMaxReduced rows (then the
// sequential sweep runs).
struct TriPlan {
  int levels;
  bool blocked;
  int64_t n[kTriMaxLevels];
  int64_t ld[kTriMaxLevels];
  int64_t off[kTriMaxLevels];
  int64_t total;
};
TriPlan tri_plan(int64_t nh);
bool tridiag_supported(const Grid& g, const Stencil& K, const Stencil& M);
// doubles of the elimination factors of Kx and Mx that tridiag_factor writes
int64_t tridiag_factor_doubles(int64_t nh);
void tridiag_factor(const Grid& g, const Stencil& K, const Stencil& M, double* fac,
                    hipStream_t st);
void tridiag_solve(const Grid& g, const Stencil& K, const Stencil& M, const int* ops, int ncols,
                   const double* const* b, double* x, int64_t ldx, const double* fac,
                   hipStream_t st);
// (Kx + s Mx) x = b, s >= 0, factors formed on the fly in work (work_doubles
// long, at least tridiag_shifted_work_doubles(Nh, ldw, ncols); the sequential
// sweep keeps ncols columns of ldw >= Nh doubles there).
int64_t tridiag_shifted_work_doubles(int64_t nh, int64_t ldw, int ncols);
void tridiag_shifted_solve(const Grid& g, const Stencil& K, const Stencil& M, double s, int ncols,
                           const double* const* b, double* x, int64_t ldx, double* work,
                           int64_t ldw, int64_t work_doubles, hipStream_t st);

// ---------------------------------------------------------------------------
// direct Mx solves for the 3-D trilinear (tensor-product) mass, tensor_mass.hip
// ---------------------------------------------------------------------------
bool tensor_mass_supported(const Grid& g, const Stencil& M);
void tensor_mass_factor(int n, double* fac, hipStream_t st);   // fac: 2 n doubles
void tensor_mass_solve(const Grid& g, const Stencil& M, int ncols, const double* const* b,
                       double* x, int64_t ldx, const double* fac, hipStream_t st);

// ---------------------------------------------------------------------------
// problem hooks for the executors (pool.hip)
// ---------------------------------------------------------------------------
// Run f, mapping library exceptions to a status and the calling thread's
// last-error message.
sts_status guarded(const std::function<void()>& f);
hipStream_t problem_stream(const sts_problem* P);
// Make s the problem's stream after the work queued on its current stream
// has finished.
void problem_bind_stream(sts_problem* P, hipStream_t s);
// Relative cost estimate of a solve (for largest-first scheduling).
double problem_cost(const sts_problem* P);
// Device bytes a problem holds after sts_create and the first capacity an
// sts_solve with this max_outer allocates (upper estimate); the basis then
// grows with the space.
int64_t problem_footprint(const sts_space& space, int64_t nt, int p, int max_outer,
                          bool mixed = false);
// Extra device bytes of `cols` more basis columns.
int64_t problem_growth_bytes(const sts_space& space, int64_t nt, int p, int64_t cols);
// Called with the extra bytes before the problem's basis grows; may block
// (to wait for memory) or throw (the solve then fails with that error).
void problem_set_grow_hook(sts_problem* P, std::function<void(int64_t)> hook);

}  // namespace sts
