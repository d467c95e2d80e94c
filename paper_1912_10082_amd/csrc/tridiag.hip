// Direct inner solves for 1-D P1 spaces.
//
// In one space dimension the P1 stiffness and mass matrices of Sec. 3 are
// constant-coefficient symmetric tridiagonal matrices, Kx = (mu / h)
// tridiag(-1, 2, -1) and Mx = (h / 6) tridiag(1, 4, 1), both symmetric positive
// definite, so Gaussian elimination without pivoting is backward stable in
// any symmetric ordering of the unknowns.  The inner solves of the extended
// Krylov space (Sec. 4) are then exact to rounding instead of an iteration
// whose count grows like 1/h.
//
// Ordering.  One sweep of the Thomas algorithm is a chain of Nh dependent
// steps; on a GPU that chain, not the memory traffic, sets the time (tens of
// milliseconds at Nh = 64k).  The unknowns are therefore ordered as in one
// level of nested dissection: every kTriPeriod-th row (63, 127, ...) is a
// separator, and the rows between two separators form an independent block
// of at most 64 rows.  For A x = d with A = tridiag(E, D, E):
//   down   each block k solves its own Dirichlet problem A_k y = d_k (a
//          Thomas sweep of <= 64 steps, all blocks and columns at once);
//   reduce the separators obey a tridiagonal system T z = r, the Schur
//          complement of the blocks:
//            T_ss   = D - E^2 (A_s^-1)_last,last - E^2 (A_{s+1}^-1)_first,first
//            T_s,s+1 = -E E (A_{s+1}^-1)_first,last
//            r_s    = d_s - E y_s,last - E y_{s+1},first,
//          again symmetric positive definite and tridiagonal, so it is solved
//          by the same scheme, recursively, until one block remains;
//   up     x_k = y_k - E z_{s-1} g_k - E z_s h_k with g_k, h_k the first and
//          last columns of A_k^-1, every row at once.
// This is Gaussian elimination in the dissection order, so it keeps the
// stability of the sequential sweep.  The pivots of every block, g_k, h_k and
// the coefficients of every reduced level depend on the matrix only: they are
// formed once per operator on the device (tri_setup_*), for Kx and Mx at
// problem set-up and for Kx + s Mx (rational Krylov, Sec. 4) per shift.  A
// solve is three launches: the down sweep of the full grid (one thread per
// block and column), every reduced level of a column inside one work-group's
// LDS (the first reduced level has at most kTriMaxReduced rows, Nh up to
// about 262k), and the up correction of the full grid.  Longer grids keep
// the sequential sweep (one thread per column).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sts_internal.h"

namespace sts {

namespace {

constexpr int kL = kTriPeriod;

// rows 63, 127, ... up to Nh - 2 are separators, so the last block is never empty
__host__ __device__ inline int64_t tri_seps(int64_t n) {
  return n >= kL + 1 ? (n - kL - 1) / kL + 1 : 0;
}

// per level: D, E (E[i] couples rows i and i + 1), the block pivots as
// m = 1 / u, al_i = E_{i-1} m_i (0 on a block's first row), c_i = E_i m_i (0
// on a block's last row), and g / h: first / last column of the block's inverse
enum { kD = 0, kE, kM, kAl, kC, kG, kH, kArrays };

__global__ void tri_fill0_kernel(double* D, double* E, int64_t n, double d, double e) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    D[i] = d;
    E[i] = e;
  }
}

// one thread per block of one level
__global__ void tri_setup_blocks_kernel(double* q, int64_t n, int64_t ld) {
  const int64_t S = tri_seps(n);
  const int64_t k = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (k > S) return;
  const double* D = q + kD * ld;
  const double* E = q + kE * ld;
  double* m = q + kM * ld;
  double* al = q + kAl * ld;
  double* c = q + kC * ld;
  double* g = q + kG * ld;
  double* h = q + kH * ld;
  const int64_t first = k * kL, end = k < S ? first + kL - 1 : n;
  double cp = 0.0;
  for (int64_t i = first; i < end; ++i) {
    const double u = i == first ? D[i] : D[i] - E[i - 1] * cp;
    const double mi = 1.0 / u;
    m[i] = mi;
    al[i] = i == first ? 0.0 : E[i - 1] * mi;
    cp = i + 1 < end ? E[i] * mi : 0.0;
    c[i] = cp;
  }
  // g = A_k^-1 e_first: forward sweep of a unit first entry, then back substitution
  double y = 0.0;
  for (int64_t i = first; i < end; ++i) {
    y = i == first ? m[i] : -al[i] * y;
    g[i] = y;
  }
  double z = 0.0;
  for (int64_t i = end - 1; i >= first; --i) {
    z = g[i] - c[i] * z;
    g[i] = z;
  }
  // h = A_k^-1 e_last: the forward sweep is zero up to the last row
  z = 0.0;
  for (int64_t i = end - 1; i >= first; --i) {
    z = i == end - 1 ? m[i] : -c[i] * z;
    h[i] = z;
  }
}

// one thread per separator: the next level's D and E (the Schur complement)
__global__ void tri_setup_next_kernel(const double* q, int64_t n, int64_t ld, double* q1,
                                      int64_t ld1) {
  const int64_t S = tri_seps(n);
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= S) return;
  const double* D = q + kD * ld;
  const double* E = q + kE * ld;
  const double* g = q + kG * ld;
  const double* h = q + kH * ld;
  const int64_t r = s * kL + kL - 1;
  const double el = E[r - 1], er = E[r];
  q1[kD * ld1 + s] = D[r] - el * el * h[r - 1] - er * er * g[r + 1];
  // block s + 1 is full (63 rows) when separator s + 1 exists
  q1[kE * ld1 + s] = s + 1 < S ? -er * E[r + kL - 1] * h[r + 1] : 0.0;
}

struct TriSolveArgs {
  TriPlan plan;
  int ncols;
  const double* base[kMaxCols];   // factor arrays of the column's operator
  const double* b[kMaxCols];
  double* x;
  int64_t ldx;
};

// level 0, one thread per (block, column): x_k = A_k^-1 d_k on the block rows
__global__ void tri_down0_kernel(TriSolveArgs a) {
  const int64_t n = a.plan.n[0], S = tri_seps(n), nb = S + 1;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = (int)(t / nb);
  if (j >= a.ncols) return;
  const int64_t k = t - (int64_t)j * nb;
  const int64_t ld = a.plan.ld[0];
  const double* q = a.base[j] + a.plan.off[0];
  const double* m = q + kM * ld;
  const double* al = q + kAl * ld;
  const double* c = q + kC * ld;
  const double* d = a.b[j];
  double* x = a.x + (int64_t)j * a.ldx;
  const int64_t first = k * kL, end = k < S ? first + kL - 1 : n;
  double y = 0.0;
#pragma unroll 8
  for (int64_t i = first; i < end; ++i) {
    y = d[i] * m[i] - al[i] * y;
    x[i] = y;
  }
  double z = 0.0;
#pragma unroll 8
  for (int64_t i = end - 1; i >= first; --i) {
    z = x[i] - c[i] * z;
    x[i] = z;
  }
}

// Every reduced level of one column in LDS (work-group j = column j): the
// level-1 right-hand side from the level-0 down sweep, down sweeps to the
// last level, up corrections back to level 1, and the level-1 solution
// written to the level-0 separator rows.
__global__ __launch_bounds__(256) void tri_reduced_kernel(TriSolveArgs a) {
  extern __shared__ double xs[];
  const int j = blockIdx.x;
  const TriPlan& p = a.plan;
  const double* base = a.base[j];
  double* x = a.x + (int64_t)j * a.ldx;
  {
    const double* E0 = base + p.off[0] + kE * p.ld[0];
    const double* d = a.b[j];
    for (int64_t s = threadIdx.x; s < p.n[1]; s += 256) {
      const int64_t r = s * kL + kL - 1;
      xs[s] = d[r] - E0[r - 1] * x[r - 1] - E0[r] * x[r + 1];
    }
  }
  // level l >= 1 sits at xs + n_1 + ... + n_{l-1}
  auto lds_off = [&](int l) {
    int64_t o = 0;
    for (int i = 1; i < l; ++i) o += p.n[i];
    return o;
  };
  __syncthreads();
  for (int l = 1; l < p.levels; ++l) {
    const int64_t n = p.n[l], S = tri_seps(n), ld = p.ld[l];
    const double* q = base + p.off[l];
    const double* m = q + kM * ld;
    const double* al = q + kAl * ld;
    const double* c = q + kC * ld;
    double* v = xs + lds_off(l);
    for (int64_t k = threadIdx.x; k <= S; k += 256) {
      const int64_t first = k * kL, end = k < S ? first + kL - 1 : n;
      double y = 0.0;
      for (int64_t i = first; i < end; ++i) {
        y = v[i] * m[i] - al[i] * y;
        v[i] = y;
      }
      double z = 0.0;
      for (int64_t i = end - 1; i >= first; --i) {
        z = v[i] - c[i] * z;
        v[i] = z;
      }
    }
    __syncthreads();
    if (l + 1 < p.levels) {
      const double* E = q + kE * ld;
      double* w = v + n;
      for (int64_t s = threadIdx.x; s < S; s += 256) {
        const int64_t r = s * kL + kL - 1;
        w[s] = v[r] - E[r - 1] * v[r - 1] - E[r] * v[r + 1];
      }
      __syncthreads();
    }
  }
  for (int l = p.levels - 2; l >= 1; --l) {
    const int64_t n = p.n[l], S = tri_seps(n), ld = p.ld[l];
    const double* q = base + p.off[l];
    double* v = xs + lds_off(l);
    const double* w = v + n;
    for (int64_t s = threadIdx.x; s < S; s += 256) v[s * kL + kL - 1] = w[s];
    __syncthreads();
    const double* E = q + kE * ld;
    const double* g = q + kG * ld;
    const double* h = q + kH * ld;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
      const int64_t k = i / kL, first = k * kL;
      if (k < S && i - first == kL - 1) continue;   // separator
      double corr = 0.0;
      if (k > 0) corr += E[first - 1] * v[first - 1] * g[i];
      if (k < S) corr += E[first + kL - 2] * v[first + kL - 1] * h[i];
      v[i] -= corr;
    }
    __syncthreads();
  }
  for (int64_t s = threadIdx.x; s < p.n[1]; s += 256) x[s * kL + kL - 1] = xs[s];
}

// level 0, one thread per (row, column): the separator correction of the block rows
__global__ void tri_up0_kernel(TriSolveArgs a) {
  const int64_t n = a.plan.n[0], S = tri_seps(n), ld = a.plan.ld[0];
  const int64_t total = n * a.ncols;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * 256) {
    const int j = (int)(t / n);
    const int64_t i = t - (int64_t)j * n;
    const int64_t k = i / kL, first = k * kL;
    if (k < S && i - first == kL - 1) continue;
    const double* q = a.base[j] + a.plan.off[0];
    const double* E = q + kE * ld;
    double* x = a.x + (int64_t)j * a.ldx;
    double corr = 0.0;
    if (k > 0) corr += E[first - 1] * x[first - 1] * q[kG * ld + i];
    if (k < S) corr += E[first + kL - 2] * x[first + kL - 1] * q[kH * ld + i];
    x[i] -= corr;
  }
}

// ---------------------------------------------------------------------------
// sequential sweeps, for grids whose first reduced level does not fit in LDS
// ---------------------------------------------------------------------------

// fac: [c_K (n) | m_K (n) | c_M (n) | m_M (n)]; thread 0 factors Kx, thread 1 Mx.
__global__ void tridiag_factor_kernel(int64_t n, double aK, double bK, double aM, double bM,
                                      double* fac) {
  const int t = threadIdx.x;
  if (t > 1) return;
  const double a = t == 0 ? aK : aM, b = t == 0 ? bK : bM;
  double* c = fac + (int64_t)t * 2 * n;
  double* m = c + n;
  double cp = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double mi = 1.0 / (b - a * cp);
    cp = a * mi;
    m[i] = mi;
    c[i] = cp;
  }
}

struct TriArgs {
  int64_t n;
  int ncols;
  int op[kMaxCols];
  const double* b[kMaxCols];
  double* x;
  int64_t ldx;
  double aK, aM;
  const double* fac;
};

__global__ void tridiag_solve_kernel(TriArgs t) {
  const int j = threadIdx.x;
  if (j >= t.ncols) return;
  const int64_t n = t.n;
  const bool k = t.op[j] == STS_OP_K;
  const double a = k ? t.aK : t.aM;
  const double* c = t.fac + (k ? 0 : 2 * n);
  const double* m = c + n;
  const double* d = t.b[j];
  double* x = t.x + (int64_t)j * t.ldx;
  double y = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    y = (d[i] - a * y) * m[i];
    x[i] = y;
  }
  double z = 0.0;
  for (int64_t i = n - 1; i >= 0; --i) {
    z = x[i] - c[i] * z;
    x[i] = z;
  }
}

// (Kx + s Mx) x = d with the factors formed during the forward sweep; the
// c_i of column j are kept in work[j * ldw ..] for the backward sweep.
__global__ void tridiag_shifted_kernel(TriArgs t, double s, double bK, double bM, double* work,
                                       int64_t ldw) {
  const int j = threadIdx.x;
  if (j >= t.ncols) return;
  const int64_t n = t.n;
  const double a = t.aK + s * t.aM, bd = bK + s * bM;
  const double* d = t.b[j];
  double* x = t.x + (int64_t)j * t.ldx;
  double* c = work + (int64_t)j * ldw;
  double y = 0.0, cp = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double mi = 1.0 / (bd - a * cp);
    cp = a * mi;
    c[i] = cp;
    y = (d[i] - a * y) * mi;
    x[i] = y;
  }
  double z = 0.0;
  for (int64_t i = n - 1; i >= 0; --i) {
    z = x[i] - c[i] * z;
    x[i] = z;
  }
}

// factor arrays of tridiag(e, d, e) for every level of the plan, at q
void tri_setup(const TriPlan& p, double d, double e, double* q, hipStream_t st) {
  const int64_t n0 = p.n[0];
  tri_fill0_kernel<<<(unsigned)std::min<int64_t>((n0 + 255) / 256, 1024), 256, 0, st>>>(
      q + p.off[0] + kD * p.ld[0], q + p.off[0] + kE * p.ld[0], n0, d, e);
  STS_HIP(hipGetLastError());
  for (int l = 0; l < p.levels; ++l) {
    const int64_t S = tri_seps(p.n[l]);
    tri_setup_blocks_kernel<<<(unsigned)((S + 1 + 63) / 64), 64, 0, st>>>(q + p.off[l], p.n[l],
                                                                          p.ld[l]);
    STS_HIP(hipGetLastError());
    if (l + 1 < p.levels) {
      tri_setup_next_kernel<<<(unsigned)((S + 255) / 256), 256, 0, st>>>(
          q + p.off[l], p.n[l], p.ld[l], q + p.off[l + 1], p.ld[l + 1]);
      STS_HIP(hipGetLastError());
    }
  }
}

void tri_blocked_solve(const TriPlan& p, int ncols, const double* const* base,
                       const double* const* b, double* x, int64_t ldx, hipStream_t st) {
  TriSolveArgs a{};
  a.plan = p;
  a.ncols = ncols;
  for (int j = 0; j < ncols; ++j) {
    a.base[j] = base[j];
    a.b[j] = b[j];
  }
  a.x = x;
  a.ldx = ldx;
  const int64_t n = p.n[0];
  const int64_t threads = (tri_seps(n) + 1) * ncols;
  // reads d, writes x, reads and writes x again
  launch(STS_K_TRIDIAG_SOLVE, 32.0 * (double)n * ncols, tri_down0_kernel,
         dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, a);
  if (p.levels > 1) {
    int64_t red = 0;
    for (int l = 1; l < p.levels; ++l) red += p.n[l];
    launch(STS_K_TRIDIAG_SOLVE, 24.0 * (double)p.n[1] * ncols, tri_reduced_kernel,
           dim3((unsigned)ncols), dim3(256), (unsigned)(red * 8), st, a);
    // reads x at the row and its separators, writes x
    const int64_t blocks = std::min<int64_t>((n * ncols + 255) / 256, 4096);
    launch(STS_K_TRIDIAG_SOLVE, 16.0 * (double)n * ncols, tri_up0_kernel,
           dim3((unsigned)blocks), dim3(256), 0, st, a);
  }
  STS_HIP(hipGetLastError());
}

}  // namespace

TriPlan tri_plan(int64_t n) {
  TriPlan p{};
  int64_t cur = std::max<int64_t>(n, 1), off = 0;
  while (p.levels < kTriMaxLevels) {
    p.n[p.levels] = cur;
    p.ld[p.levels] = (cur + 31) / 32 * 32;
    p.off[p.levels] = off;
    off += kArrays * p.ld[p.levels];
    ++p.levels;
    const int64_t s = tri_seps(cur);
    if (s == 0) break;
    cur = s;
  }
  p.total = off;
  p.blocked = tri_seps(p.n[p.levels - 1]) == 0 && (p.levels == 1 || p.n[1] <= kTriMaxReduced);
  return p;
}

int64_t tridiag_factor_doubles(int64_t nh) {
  const TriPlan p = tri_plan(nh);
  return p.blocked ? 2 * p.total : 4 * nh;
}

int64_t tridiag_shifted_work_doubles(int64_t nh, int64_t ldw, int ncols) {
  const TriPlan p = tri_plan(nh);
  return p.blocked ? p.total : ldw * ncols;
}

void tridiag_shifted_solve(const Grid& g, const Stencil& K, const Stencil& M, double s, int ncols,
                           const double* const* b, double* x, int64_t ldx, double* work,
                           int64_t ldw, int64_t work_doubles, hipStream_t st) {
  STS_REQUIRE(ncols >= 0 && ncols <= kMaxCols, STS_E_INVALID, "tridiagonal solve: 0..8 columns");
  STS_REQUIRE(s >= 0.0, STS_E_INVALID, "tridiagonal solve: shift must be >= 0");
  if (ncols == 0 || g.nh <= 0) return;
  const TriPlan p = tri_plan(g.nh);
  STS_REQUIRE(work_doubles >= tridiag_shifted_work_doubles(g.nh, ldw, ncols), STS_E_INVALID,
              "tridiagonal solve: work too small");
  if (p.blocked) {
    // the shifted matrix's factors, then the blocked solve
    tri_setup(p, K.c[13] + s * M.c[13], K.c[12] + s * M.c[12], work, st);
    const double* base[kMaxCols];
    for (int j = 0; j < ncols; ++j) base[j] = work;
    tri_blocked_solve(p, ncols, base, b, x, ldx, st);
    return;
  }
  STS_REQUIRE(ldw >= g.nh, STS_E_INVALID, "tridiagonal solve: work too small");
  TriArgs t{};
  t.n = g.nh;
  t.ncols = ncols;
  for (int j = 0; j < ncols; ++j) {
    t.op[j] = STS_OP_K;
    t.b[j] = b[j];
  }
  t.x = x;
  t.ldx = ldx;
  t.aK = K.c[12];
  t.aM = M.c[12];
  // reads b, writes c and x, reads c and x, writes x
  launch(STS_K_TRIDIAG_SOLVE, 48.0 * (double)g.nh * ncols, tridiag_shifted_kernel, dim3(1),
         dim3(64), 0, st, t, s, K.c[13], M.c[13], work, ldw);
  STS_HIP(hipGetLastError());
}

bool tridiag_supported(const Grid& g, const Stencil& K, const Stencil& M) {
  if (g.dim != 1) return false;
  // only the x-neighbours (indices 12, 14 of the 27-point numbering) and the centre
  for (int i = 0; i < 27; ++i) {
    if (i == 12 || i == 13 || i == 14) continue;
    if (K.c[i] != 0.0 || M.c[i] != 0.0) return false;
  }
  return K.c[12] == K.c[14] && M.c[12] == M.c[14] && K.c[13] > 0.0 && M.c[13] > 0.0;
}

void tridiag_factor(const Grid& g, const Stencil& K, const Stencil& M, double* fac,
                    hipStream_t st) {
  const TriPlan p = tri_plan(g.nh);
  if (p.blocked) {
    tri_setup(p, K.c[13], K.c[12], fac, st);
    tri_setup(p, M.c[13], M.c[12], fac + p.total, st);
    return;
  }
  tridiag_factor_kernel<<<1, 64, 0, st>>>(g.nh, K.c[12], K.c[13], M.c[12], M.c[13], fac);
  STS_HIP(hipGetLastError());
}

void tridiag_solve(const Grid& g, const Stencil& K, const Stencil& M, const int* ops, int ncols,
                   const double* const* b, double* x, int64_t ldx, const double* fac,
                   hipStream_t st) {
  STS_REQUIRE(ncols >= 0 && ncols <= kMaxCols, STS_E_INVALID, "tridiagonal solve: 0..8 columns");
  if (ncols == 0 || g.nh <= 0) return;
  const TriPlan p = tri_plan(g.nh);
  if (p.blocked) {
    const double* base[kMaxCols];
    for (int j = 0; j < ncols; ++j) base[j] = fac + (ops[j] == STS_OP_K ? 0 : p.total);
    tri_blocked_solve(p, ncols, base, b, x, ldx, st);
    return;
  }
  TriArgs t{};
  t.n = g.nh;
  t.ncols = ncols;
  for (int j = 0; j < ncols; ++j) {
    t.op[j] = ops[j];
    t.b[j] = b[j];
  }
  t.x = x;
  t.ldx = ldx;
  t.aK = K.c[12];
  t.aM = M.c[12];
  t.fac = fac;
  // each column reads b once and reads / writes x twice
  launch(STS_K_TRIDIAG_SOLVE, 32.0 * (double)g.nh * ncols, tridiag_solve_kernel, dim3(1),
         dim3(64), 0, st, t);
  STS_HIP(hipGetLastError());
}

}  // namespace sts
