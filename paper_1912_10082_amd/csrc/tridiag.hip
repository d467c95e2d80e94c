// Direct inner solves for 1-D P1 spaces.
//
// In one space dimension the P1 stiffness and mass matrices of Sec. 3 are
// constant-coefficient symmetric tridiagonal matrices, Kx = (mu / h)
// tridiag(-1, 2, -1) and Mx = (h / 6) tridiag(1, 4, 1), both symmetric positive
// definite and (weakly) diagonally dominant, so Gaussian elimination without
// pivoting (the Thomas algorithm) is backward stable.  The elimination
// factors depend only on the matrix: for A = tridiag(a, b, a) of order n,
//   m_0 = 1 / b,  m_i = 1 / (b - a c_{i-1}),  c_i = a m_i,
// computed once per operator (tridiag_factor_kernel).  A solve is then
//   y_0 = d_0 m_0,  y_i = (d_i - a y_{i-1}) m_i       (forward)
//   x_{n-1} = y_{n-1},  x_i = y_i - c_i x_{i+1}        (backward),
// one thread per right-hand side, two sequential sweeps of n steps whose
// dependent chain is one fused multiply-add per step.  The inner solves of
// the extended Krylov space (Sec. 4) are then exact to rounding instead of
// an iteration whose count grows like 1/h.
#include <hip/hip_runtime.h>

#include "sts_internal.h"

namespace sts {

namespace {

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

}  // namespace

void tridiag_shifted_solve(const Grid& g, const Stencil& K, const Stencil& M, double s, int ncols,
                           const double* const* b, double* x, int64_t ldx, double* work,
                           int64_t ldw, hipStream_t st) {
  STS_REQUIRE(ncols >= 0 && ncols <= kMaxCols, STS_E_INVALID, "tridiagonal solve: 0..8 columns");
  STS_REQUIRE(s >= 0.0, STS_E_INVALID, "tridiagonal solve: shift must be >= 0");
  if (ncols == 0 || g.nh <= 0) return;
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
  tridiag_factor_kernel<<<1, 64, 0, st>>>(g.nh, K.c[12], K.c[13], M.c[12], M.c[13], fac);
  STS_HIP(hipGetLastError());
}

void tridiag_solve(const Grid& g, const Stencil& K, const Stencil& M, const int* ops, int ncols,
                   const double* const* b, double* x, int64_t ldx, const double* fac,
                   hipStream_t st) {
  STS_REQUIRE(ncols >= 0 && ncols <= kMaxCols, STS_E_INVALID, "tridiagonal solve: 0..8 columns");
  if (ncols == 0 || g.nh <= 0) return;
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
