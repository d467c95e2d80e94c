// Triangular factor of a tall matrix by blocked Householder QR.
//
// The exact residual of the Galerkin solution (Sec. 4: the Sylvester
// residual of U = V Y) is R = A B^T with A = [F1, Kx V, Mx V] (Nh x n) and
// B = [F2, -Mt Y^T, -Dt Y^T] (Nt x n), n = P + 2k.  For any factorisation
// B = Q_B R_B with orthonormal columns in Q_B, ||A B^T||_F = ||A R_B^T||_F:
// when Nt is well above n this replaces the Nh x n x Nt product by an
// Nh x n x n one.  Householder QR is columnwise backward stable
// (B + E = Q_B R_B with ||e_j|| = O(eps) ||b_j||), so the norm's rounding
// error is of the order of the direct product's.
//
// Blocked algorithm, panels of kQrNb columns:
//  - the panel is factored by one work-group of 1024 threads holding the
//    panel in registers (rows <= 1024 RPT): per column a Householder
//    reflector (LAPACK's dlarfg convention: H = I - tau v v^T, v_0 = 1,
//    H x = beta e_0) and its application to the panel's later columns, and
//    the triangular factor T of the compact form H_0 ... H_{nb-1} = I - V T V^T;
//  - the trailing columns get Q^T = I - V T^T V^T: C = A^T V (the tall-skinny
//    Gram kernel), then A -= V (T^T C^T) in one streaming launch.
// Only the upper triangle (R) of the result is used.
#include <hip/hip_runtime.h>

#include <cmath>

#include "sts_internal.h"

namespace sts {

namespace {

constexpr int kQrT = 1024;   // threads of the panel kernel
constexpr int kQrW = kQrT / 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums over the work-group of NV values per thread (fixed order); the totals
// land in out[0..NV).  Two barriers.
template <int NV>
__device__ __forceinline__ void group_sums(const double (&v)[NV], int nv, double (*red)[kQrNb],
                                           double* out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    if (j < nv) {
      const double s = wave_sum(v[j]);
      if (lane == 0) red[w][j] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    double s = 0.0;
    for (int q = 0; q < kQrW; ++q) s += red[q][threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Factor the panel A[j0.., j0..j0+nb) (rows j0..rows-1).  Writes R's rows of
// the panel back into A, the reflectors (unit diagonal, zeros above) into
// V (rows - j0 rows, ldv) and T (kQrNb x kQrNb, column-major).
template <int RPT>
__global__ __launch_bounds__(kQrT) void qr_panel_kernel(int64_t rows, int j0, int nb, double* A,
                                                        int64_t lda, double* V, int64_t ldv,
                                                        double* Tg) {
  __shared__ double red[kQrW][kQrNb];
  __shared__ double sums[kQrNb];
  __shared__ double piv[kQrNb];
  __shared__ double T[kQrNb][kQrNb];
  const int t = threadIdx.x;
  const int64_t L = rows - j0;
  double x[RPT][kQrNb];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int64_t rho = t + (int64_t)kQrT * i;
#pragma unroll
    for (int c = 0; c < kQrNb; ++c)
      x[i][c] = (rho < L && c < nb) ? A[(j0 + rho) + (int64_t)(j0 + c) * lda] : 0.0;
  }
  if (t < kQrNb * kQrNb) T[t / kQrNb][t % kQrNb] = 0.0;
#pragma unroll
  for (int c = 0; c < kQrNb; ++c) {
    if (c >= nb) break;
    // alpha = x[c][c] (row c is owned by thread c, i = 0), sigma = sum below
    if (t == c) piv[c] = x[0][c];
    double part[1] = {0.0};
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int64_t rho = t + (int64_t)kQrT * i;
      if (rho > c) part[0] += x[i][c] * x[i][c];
    }
    group_sums<1>(part, 1, red, sums);
    const double alpha = piv[c], sigma = sums[0];
    double tau = 0.0, beta = alpha, scale = 0.0;
    if (sigma > 0.0) {
      const double nrm = sqrt(alpha * alpha + sigma);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    // v in column c from row c down (1 at row c, x * scale below); the rows
    // above keep R's entries of column c, the diagonal goes to piv
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int64_t rho = t + (int64_t)kQrT * i;
      if (rho >= c) x[i][c] = rho > c ? x[i][c] * scale : 1.0;
    }
    // w_j = v^T x_j for the later columns; z_k = v_k^T v for the earlier ones
    double wz[kQrNb];
#pragma unroll
    for (int j = 0; j < kQrNb; ++j) wz[j] = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int64_t rho = t + (int64_t)kQrT * i;
      if (rho >= c) {
        const double vi = x[i][c];
#pragma unroll
        for (int j = 0; j < kQrNb; ++j)
          if (j != c) wz[j] += vi * x[i][j];
      }
    }
    group_sums<kQrNb>(wz, nb, red, sums);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int64_t rho = t + (int64_t)kQrT * i;
      if (rho >= c) {
        const double tv = tau * x[i][c];
#pragma unroll
        for (int j = c + 1; j < kQrNb; ++j)
          if (j < nb) x[i][j] -= tv * sums[j];
      }
    }
    if (t == 0) {
      // T[0:c, c] = -tau T[0:c, 0:c] z, T[c][c] = tau
      for (int k = 0; k < c; ++k) {
        double s = 0.0;
        for (int q = k; q < c; ++q) s += T[k][q] * sums[q];
        T[k][c] = -tau * s;
      }
      T[c][c] = tau;
      piv[c] = beta;
    }
    __syncthreads();
  }
  // write back: V (explicit), R's rows of the panel into A
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int64_t rho = t + (int64_t)kQrT * i;
    if (rho < L) {
#pragma unroll
      for (int c = 0; c < kQrNb; ++c) {
        if (c < nb) {
          V[rho + (int64_t)c * ldv] = rho >= c ? x[i][c] : 0.0;
          if (rho < c) A[(j0 + rho) + (int64_t)(j0 + c) * lda] = x[i][c];   // R above the diagonal
          if (rho == c) A[(j0 + rho) + (int64_t)(j0 + c) * lda] = piv[c];   // R's diagonal
        }
      }
    }
  }
  if (t < kQrNb * kQrNb) Tg[t] = T[t % kQrNb][t / kQrNb];
}

// A[:, 0..m) -= V (T^T C^T) on rows 0..rows-1, with C = A^T V (m x nb, ldc).
constexpr int kUpdCols = 32;
__global__ __launch_bounds__(256) void qr_update_kernel(int64_t rows, int m, int nb, double* A,
                                                        int64_t lda, const double* V, int64_t ldv,
                                                        const double* C, int64_t ldc,
                                                        const double* Tg) {
  __shared__ double G[kQrNb][kUpdCols];
  const int c0 = blockIdx.y * kUpdCols;
  const int ncol = min(kUpdCols, m - c0);
  // G[j][i] = sum_k T[k][j] C[c0 + i][k]
  for (int e = threadIdx.x; e < kQrNb * kUpdCols; e += 256) {
    const int j = e / kUpdCols, i = e % kUpdCols;
    double s = 0.0;
    if (j < nb && i < ncol)
      for (int k = 0; k <= j; ++k) s += Tg[k + j * kQrNb] * C[(c0 + i) + (int64_t)k * ldc];
    G[j][i] = s;
  }
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  double v[kQrNb];
#pragma unroll
  for (int j = 0; j < kQrNb; ++j) v[j] = j < nb ? V[r + (int64_t)j * ldv] : 0.0;
  for (int i = 0; i < ncol; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kQrNb; ++j) s += v[j] * G[j][i];
    A[r + (int64_t)(c0 + i) * lda] -= s;
  }
}

// Rc = the upper triangle of A's leading n x n block, zeros below.
__global__ void qr_copy_r_kernel(int n, const double* A, int64_t lda, double* Rc) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int r = (int)(e % n), c = (int)(e / n);
  Rc[e] = r <= c ? A[r + (int64_t)c * lda] : 0.0;
}

}  // namespace

bool qr_r_supported(int64_t rows, int n) { return n >= 1 && rows >= n && rows <= kQrMaxRows; }

size_t qr_r_work_doubles(int64_t rows, int n) {
  // V (rows x nb), C (n x nb), T (nb x nb), the Gram partials
  return (size_t)rows * kQrNb + (size_t)n * kQrNb + kQrNb * kQrNb +
         (size_t)gemm_tn_partial_size(rows, n);
}

void qr_r(int64_t rows, int n, double* A, int64_t lda, double* Rc, double* work, hipStream_t st) {
  STS_REQUIRE(qr_r_supported(rows, n), STS_E_INVALID, "qr_r: shape out of range");
  double* V = work;
  double* C = V + (size_t)rows * kQrNb;
  double* T = C + (size_t)n * kQrNb;
  double* part = T + kQrNb * kQrNb;
  for (int j0 = 0; j0 < n; j0 += kQrNb) {
    const int nb = std::min(kQrNb, n - j0);
    const int64_t L = rows - j0;
    // profiled as the residual's QR (the Gram products below count under the
    // Gram kernel)
    const double pb = 16.0 * (double)L * nb;
    if (L <= kQrT)
      launch(STS_K_RESIDUAL_QR, pb, qr_panel_kernel<1>, dim3(1), dim3(kQrT), 0, st, rows, j0, nb, A,
             lda, V, L, T);
    else if (L <= 2 * kQrT)
      launch(STS_K_RESIDUAL_QR, pb, qr_panel_kernel<2>, dim3(1), dim3(kQrT), 0, st, rows, j0, nb, A,
             lda, V, L, T);
    else
      launch(STS_K_RESIDUAL_QR, pb, qr_panel_kernel<4>, dim3(1), dim3(kQrT), 0, st, rows, j0, nb, A,
             lda, V, L, T);
    STS_HIP(hipGetLastError());
    const int m = n - j0 - nb;
    if (m <= 0) continue;
    double* At = A + j0 + (int64_t)(j0 + nb) * lda;
    gemm_tn(L, m, nb, At, lda, V, L, C, m, part, st);   // C = At^T V (m x nb)
    const dim3 grid((unsigned)((L + 255) / 256), (unsigned)((m + kUpdCols - 1) / kUpdCols));
    launch(STS_K_RESIDUAL_QR, 8.0 * (double)L * (2.0 * m + nb), qr_update_kernel, grid, dim3(256), 0,
           st, L, m, nb, At, lda, (const double*)V, L, (const double*)C, m, (const double*)T);
    STS_HIP(hipGetLastError());
  }
  qr_copy_r_kernel<<<(unsigned)(((int64_t)n * n + 255) / 256), 256, 0, st>>>(n, A, lda, Rc);
  STS_HIP(hipGetLastError());
}

}  // namespace sts
