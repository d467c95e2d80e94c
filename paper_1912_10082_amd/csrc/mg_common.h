// Device helpers shared by the 2-D and 3-D multigrid-preconditioned CG.
#pragma once

#include <hip/hip_runtime.h>

#include "sts_internal.h"

namespace sts {
namespace mgc {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the work-group (fixed order); every thread gets the result.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// g[idx] if `in`, else zero, without a branch: outside, the load reads the
// column's first element instead and the value is dropped.  A load under a
// branch sits in a basic block of its own and waits for its data before the
// next one is issued; branch-free loads of a fully unrolled loop are all in
// flight together, which is what a latency-bound tile fill needs.
template <class T>
__device__ __forceinline__ T ld_or_zero(const T* g, bool in, size_t idx) {
  const T v = g[in ? idx : 0];
  return in ? v : (T)0;
}

// A thread's share of an LDS fill of N slots by NT threads (slots
// threadIdx.x + k NT): load() issues every load into registers, store()
// writes them, so a kernel can put several fills (and its other global
// reads) in flight before the first wait.  get(i) must be branch-free (ld_or_zero); the last partial
// round re-reads slot N - 1 and drops it.
template <int N, class S, int NT>
struct StagedN {
  static constexpr int NI = (N + NT - 1) / NT;
  S v[NI];
  template <class F>
  __device__ __forceinline__ void load(F&& get) {
#pragma unroll
    for (int k = 0; k < NI; ++k) v[k] = get(min((int)threadIdx.x + k * NT, N - 1));
  }
  __device__ __forceinline__ void store(S* s) const {
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const int i = threadIdx.x + k * NT;
      if (i < N) s[i] = v[k];
    }
  }
};

// Consecutive block ids go round-robin over the 8 XCDs; give each XCD a
// contiguous range of tiles so that halo neighbours share an L2.
__device__ __forceinline__ int xcd_remap(int bid, int n) {
  const int q = n >> 3, rem = n & 7;
  const int x = bid & 7, j = bid >> 3;
  return x * q + min(x, rem) + j;
}

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64: lane l = i + 16 g supplies a = X[i][g] and
// b = Y[g][i]; element q of the accumulator is (X Y)[4 q + g][i].
__device__ __forceinline__ d4 mfma(double x, double y, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
}

// Chebyshev smoothing coefficients: d_0 = c_0 r_0 / D and, for k >= 1,
// d_k = a_k d_{k-1} + c_k r_k / D with r_k = b - K u_k; u_{k+1} = u_k + d_k.
// The coefficients of step k do not depend on the number of steps taken.
struct Smooth {
  double a[kMGNu];
  double c[kMGNu];
};

// Chebyshev coefficients for the interval [lo, 2] of the spectrum of D^{-1} Kx.
inline Smooth smooth_coefficients(double lo) {
  const double hi = 2.0;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  Smooth s{};
  double rho = 1.0 / sigma;
  s.a[0] = 0.0;
  s.c[0] = 1.0 / theta;
  for (int k = 1; k < kMGNu; ++k) {
    const double rho1 = 1.0 / (2.0 * sigma - rho);
    s.a[k] = rho1 * rho;
    s.c[k] = 2.0 * rho1 / delta;
    rho = rho1;
  }
  return s;
}

// The preconditioned-CG decision taken at the start of an iteration from
// rr = (r, r), rz = (r, z) and the previous step's alpha (0 = breakdown):
// stop (converged, iteration cap, breakdown) or continue with beta.  Every
// work-group of a column evaluates it on bitwise identical sums.
__device__ __forceinline__ bool pcg_decide(CGScal& s, double rr, double rz, double alpha_prev,
                                           double& beta) {
  bool go = false;
  beta = 0.0;
  const int done = s.iters;
  if (done > 0 && !(alpha_prev > 0.0)) {
    s.active = 0;
    s.flag = 3;   // (p, K p) was not positive or not finite
  } else if (!__builtin_isfinite(rr) || !__builtin_isfinite(rz)) {
    s.active = 0;
    s.flag = 3;
  } else if (done == 0 && rr == 0.0) {
    s.gamma0 = 0.0;
    s.active = 0;
    s.flag = 1;   // b = 0: x = 0
  } else if (done > 0 && rr <= s.rtol2 * s.gamma0) {
    s.active = 0;
    s.flag = 1;
  } else if (done >= s.maxit) {
    s.active = 0;
    s.flag = 2;
  } else if (!(rz > 0.0)) {
    s.active = 0;
    s.flag = 3;   // the preconditioner lost definiteness in rounding
  } else {
    if (done == 0) s.gamma0 = rr;
    beta = done == 0 ? 0.0 : rz / s.rho;
    s.rho = rz;
    s.iters = done + 1;
    go = true;
  }
  s.gamma = rr;
  return go;
}

}  // namespace mgc
}  // namespace sts
