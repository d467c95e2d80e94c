// The reduced (projected) problem of the Galerkin method.
//
// With an Mx-orthonormal basis V the reduced spatial pencil is (Km, I) up to
// rounding, Km = V^T Kx V.  Its eigendecomposition Km Q = Q diag(lam) turns
// the reduced Sylvester equation Km Y Mt^T + Y Dt^T = beta F2^T into k
// independent lower-bidiagonal recurrences in time, one per eigencomponent:
//   (Dt + lam_i Mt) z_i = (Q^T beta F2^T)[i, :],   Y = Q Z.
//
// This file holds the time sweep, the reduced residual and the small dense
// helpers; the eigendecomposition itself is in eig.hip.
#include <hip/hip_runtime.h>

#include <cmath>

#include "sts_internal.h"

namespace sts {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// time sweep
// ---------------------------------------------------------------------------
struct SweepArgs {
  int k, nt, p;
  const double* lam;
  const double* qb;
  int64_t ldqb;
  const double* F2;
  int64_t ldf;
  TimeOps t;
  double* Z;
  int64_t ldz;
  const double* G;   // if set: full right-hand side G (k x nt, ldg) instead of qb F2^T
  int64_t ldg;
};

// Row l of (Dt + lam Mt) z = g reads d_l z_l + c_l z_{l-1} = g_l, i.e. the
// first-order linear recurrence z_l = a_l z_{l-1} + b_l with a_l = -c_l / d_l,
// b_l = g_l / d_l (|a_l| < 1 for the Crank-Nicolson pencil, lam > 0).  A
// work-group takes kSweepI eigencomponents and cuts the time axis into
// kSweepC chunks, one thread per (component, chunk):
//   1. each thread runs its chunk from z = 0, stores that particular solution
//      and keeps the chunk's product of a_l;
//   2. one thread per component carries the values entering each chunk
//      across the kSweepC chunks;
//   3. each thread adds (running product of a_l) x (value entering its chunk).
// The dependent chain is nt / kSweepC + kSweepC steps instead of nt.
constexpr int kSweepI = 16;
constexpr int kSweepC = 16;

__global__ __launch_bounds__(kSweepI * kSweepC) void sweep_kernel(SweepArgs a) {
  __shared__ double yend[kSweepC][kSweepI], prod[kSweepC][kSweepI], zin[kSweepC][kSweepI];
  const int il = threadIdx.x % kSweepI, c = threadIdx.x / kSweepI;
  const int i = blockIdx.x * kSweepI + il;
  const bool act = i < a.k;
  const double lam = act ? a.lam[i] : 0.0;
  double q[4] = {0.0, 0.0, 0.0, 0.0};
  for (int p = 0; p < a.p; ++p) q[p] = act ? a.qb[i + p * a.ldqb] : 0.0;
  const int len = (a.nt + kSweepC - 1) / kSweepC;
  const int l0 = c * len, l1 = min(a.nt, l0 + len);
  double* Zi = a.Z + (act ? i : 0);
  auto coef = [&](int l, double& al, double& bl) {
    double g = 0.0;
    if (a.G) g = a.G[i + (int64_t)l * a.ldg];
    else
      for (int p = 0; p < a.p; ++p) g += q[p] * a.F2[l + p * a.ldf];
    const double d = a.t.d[l] + lam * a.t.m[l];
    const double cl = l > 0 ? a.t.e[l - 1] + lam * a.t.n[l - 1] : 0.0;
    al = -cl / d;
    bl = g / d;
  };
  double y = 0.0, pr = 1.0;
  if (act) {
#pragma unroll 4
    for (int l = l0; l < l1; ++l) {
      double al, bl;
      coef(l, al, bl);
      y = al * y + bl;
      pr *= al;
      Zi[(int64_t)l * a.ldz] = y;
    }
  }
  yend[c][il] = y;
  prod[c][il] = pr;
  __syncthreads();
  if (c == 0) {
    double z = 0.0;
    for (int u = 0; u < kSweepC; ++u) {
      zin[u][il] = z;
      z = yend[u][il] + prod[u][il] * z;
    }
  }
  __syncthreads();
  const double z0 = zin[c][il];
  if (act && z0 != 0.0) {
    double cum = 1.0;
#pragma unroll 4
    for (int l = l0; l < l1; ++l) {
      double al, bl;
      coef(l, al, bl);
      cum *= al;
      Zi[(int64_t)l * a.ldz] += cum * z0;
    }
  }
}

// out (nt x k, ldo) = scale * T A^T for A (k x nt) and lower-bidiagonal T:
// out[l, i] = scale (td[l] A[i, l] + ts[l-1] A[i, l-1]).
// R = beta F2^T - KY Mt^T - Y Dt^T (k x nt), KY = Km Y.  Row l of a
// lower-bidiagonal time matrix T has T[l, l] and T[l, l-1].
__global__ void reduced_residual_kernel(int k, int nt, int p, const double* beta, int64_t ldb,
                                        const double* F2, int64_t ldf, const double* KY,
                                        const double* Y, int64_t ldy, TimeOps t, double* R,
                                        int64_t ldr) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)k * nt) return;
  const int i = idx % k, l = idx / k;
  double f = 0.0;
  for (int q = 0; q < p; ++q) f += beta[i + (int64_t)q * ldb] * F2[l + (int64_t)q * ldf];
  const int64_t c = i + (int64_t)l * ldy;
  double v = f - t.m[l] * KY[c] - t.d[l] * Y[c];
  if (l > 0) v -= t.n[l - 1] * KY[c - ldy] + t.e[l - 1] * Y[c - ldy];
  R[i + (int64_t)l * ldr] = v;
}

__global__ void bidiag_right_kernel(int k, int nt, const double* A, int64_t lda, const double* td,
                                    const double* ts, double scale, double* out, int64_t ldo) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)k * nt) return;
  const int l = idx % nt, i = idx / nt;
  double v = td[l] * A[i + (int64_t)l * lda];
  if (l > 0) v += ts[l - 1] * A[i + (int64_t)(l - 1) * lda];
  out[l + (int64_t)i * ldo] = scale * v;
}

__global__ void transpose_kernel(int m, int n, const double* A, int64_t lda, double* B,
                                 int64_t ldb) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * n) return;
  const int j = idx % n, i = idx / n;
  B[j + (int64_t)i * ldb] = A[i + (int64_t)j * lda];
}

__global__ void chol_lower_kernel(int b, const double* G, int64_t ldg, double* L, int64_t ldl,
                                  int* ok) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int good = 1;
  for (int j = 0; j < b; ++j)
    for (int i = 0; i < b; ++i) L[i + j * ldl] = 0.0;
  for (int j = 0; j < b; ++j) {
    double d = G[j + j * ldg];
    for (int q = 0; q < j; ++q) d -= L[j + q * ldl] * L[j + q * ldl];
    if (!(d > 0.0)) {
      good = 0;
      d = 0.0;
    }
    const double ljj = sqrt(d);
    L[j + j * ldl] = ljj;
    for (int i = j + 1; i < b; ++i) {
      double s = G[i + j * ldg];
      for (int q = 0; q < j; ++q) s -= L[i + q * ldl] * L[j + q * ldl];
      L[i + j * ldl] = ljj > 0.0 ? s / ljj : 0.0;
    }
  }
  *ok = good;
}

// dst[c, r] = src[r, c] for r < m, c < n (dst is n x m, ldd)
__global__ void mirror_kernel(int m, int n, const double* src, int64_t lds, double* dst,
                              int64_t ldd) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * n) return;
  const int r = idx % m, c = idx / m;
  dst[c + (int64_t)r * ldd] = src[r + (int64_t)c * lds];
}

// ||L^T (m_l T1[:, l] + n_{l-1} T1[:, l-1])||^2 summed over l.
__global__ __launch_bounds__(256) void cheap_res_kernel(int b, int nt, const double* T1,
                                                        int64_t ldt, const double* L, int64_t ldl,
                                                        const double* md, const double* ms,
                                                        double* partial, unsigned* counter,
                                                        double* out) {
  __shared__ double red[4];
  __shared__ int last;
  const int l = blockIdx.x * 256 + threadIdx.x;
  double s = 0.0;
  if (l < nt) {
    double vv[16];
    for (int r = 0; r < b; ++r) {
      double x = md[l] * T1[r + (int64_t)l * ldt];
      if (l > 0) x += ms[l - 1] * T1[r + (int64_t)(l - 1) * ldt];
      vv[r] = x;
    }
    for (int c = 0; c < b; ++c) {   // (L^T v)_c = sum_{r >= c} L[r, c] v_r
      double u = 0.0;
      for (int r = c; r < b; ++r) u += L[r + c * ldl] * vv[r];
      s += u * u;
    }
  }
  s = wave_sum(s);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    __threadfence();
    last = atomicAdd(counter, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double t = 0.0;
  for (int q = threadIdx.x; q < (int)gridDim.x; q += 256) t += partial[q];
  t = wave_sum(t);
  __syncthreads();
  if (lane == 0) red[wv] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    *out = (red[0] + red[1]) + (red[2] + red[3]);
    atomicExch(counter, 0u);
  }
}

}  // namespace


void time_sweep(int k, int nt, int p, const double* lam, const double* qb, int64_t ldqb,
                const double* F2, int64_t ldf, const TimeOps& t, double* Z, int64_t ldz,
                hipStream_t st) {
  if (k <= 0 || nt <= 0) return;
  STS_REQUIRE(p >= 1 && p <= 4, STS_E_INVALID, "time_sweep: 1 <= p <= 4");
  SweepArgs a{k, nt, p, lam, qb, ldqb, F2, ldf, t, Z, ldz, nullptr, 0};
  launch(STS_K_SWEEP, 8.0 * (double)k * nt, sweep_kernel, dim3((k + kSweepI - 1) / kSweepI),
         dim3(kSweepI * kSweepC), 0, st, a);
  STS_HIP(hipGetLastError());
}

void time_sweep_full(int k, int nt, const double* lam, const double* G, int64_t ldg,
                     const TimeOps& t, double* Z, int64_t ldz, hipStream_t st) {
  if (k <= 0 || nt <= 0) return;
  SweepArgs a{k, nt, 0, lam, nullptr, 0, nullptr, 0, t, Z, ldz, G, ldg};
  launch(STS_K_SWEEP, 8.0 * (double)k * nt, sweep_kernel, dim3((k + kSweepI - 1) / kSweepI),
         dim3(kSweepI * kSweepC), 0, st, a);
  STS_HIP(hipGetLastError());
}

void reduced_residual(int k, int nt, int p, const double* beta, int64_t ldb, const double* F2,
                      int64_t ldf, const double* KY, const double* Y, int64_t ldy,
                      const TimeOps& t, double* R, int64_t ldr, hipStream_t st) {
  if (k <= 0 || nt <= 0) return;
  const int64_t n = (int64_t)k * nt;
  reduced_residual_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(k, nt, p, beta, ldb, F2,
                                                                       ldf, KY, Y, ldy, t, R, ldr);
  STS_HIP(hipGetLastError());
}

void bidiag_right(int k, int nt, const double* A, int64_t lda, const double* td, const double* ts,
                  double scale, double* out, int64_t ldo, hipStream_t st) {
  const int64_t n = (int64_t)k * nt;
  if (n <= 0) return;
  bidiag_right_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(k, nt, A, lda, td, ts, scale,
                                                                    out, ldo);
  STS_HIP(hipGetLastError());
}

void transpose(int m, int n, const double* A, int64_t lda, double* B, int64_t ldb,
               hipStream_t st) {
  const int64_t cnt = (int64_t)m * n;
  if (cnt <= 0) return;
  transpose_kernel<<<(unsigned)((cnt + 255) / 256), 256, 0, st>>>(m, n, A, lda, B, ldb);
  STS_HIP(hipGetLastError());
}

void chol_lower(int b, const double* G, int64_t ldg, double* L, int64_t ldl, int* ok,
                hipStream_t st) {
  chol_lower_kernel<<<1, 64, 0, st>>>(b, G, ldg, L, ldl, ok);
  STS_HIP(hipGetLastError());
}

void mirror(int m, int n, const double* src, int64_t lds, double* dst, int64_t ldd,
            hipStream_t st) {
  const int64_t cnt = (int64_t)m * n;
  if (cnt <= 0) return;
  mirror_kernel<<<(unsigned)((cnt + 255) / 256), 256, 0, st>>>(m, n, src, lds, dst, ldd);
  STS_HIP(hipGetLastError());
}

void cheap_residual(int b, int nt, const double* T1, int64_t ldt, const double* L, int64_t ldl,
                    const double* md, const double* ms, double* out, double* partial,
                    unsigned* counter, hipStream_t st) {
  STS_REQUIRE(b >= 1 && b <= 16, STS_E_INVALID, "cheap_residual: 1 <= b <= 16");
  const int blocks = (nt + 255) / 256;
  cheap_res_kernel<<<blocks, 256, 0, st>>>(b, nt, T1, ldt, L, ldl, md, ms, partial, counter, out);
  STS_HIP(hipGetLastError());
}

}  // namespace sts
