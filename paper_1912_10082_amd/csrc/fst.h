// Radix-2 FFT building blocks in LDS for the fast sine transforms of the
// exact coarse-grid solves (2-D in mg.hip, 3-D in mg3.hip).
//
// The raw sine transform y_k = sum_{j=1..m} x_j sin(pi j k / L), L = m + 1 a
// power of two, is -1/2 Im of the length-2L discrete Fourier transform of the
// odd extension (0, x_1 .. x_m, 0, -x_m .. -x_1); two real vectors share one
// complex transform of x1 + i x2 (y1 = -Im Z / 2, y2 = Re Z / 2).  A work-group
// of L threads runs one transform, one butterfly per thread per stage.
#pragma once

#include <hip/hip_runtime.h>

namespace sts {

template <int L>
struct FftBits {
  static constexpr int value = L == 8 ? 4 : L == 16 ? 5 : L == 32 ? 6 : L == 64 ? 7
                               : L == 128 ? 8 : 9;
  static_assert(L == 8 || L == 16 || L == 32 || L == 64 || L == 128 || L == 256,
                "transform lengths 2L with L = 8 .. 256");
};

// In-place FFT of N = 2L complex values held in bit-reversed order; tw holds
// cos, sin of pi k / L for k < L.
template <int L>
__device__ __forceinline__ void fft_lds(double2* z, const double* tw) {
  constexpr int N = 2 * L;
  const int b = threadIdx.x;
#pragma unroll
  for (int h = 1; h < N; h <<= 1) {
    const int j = b & (h - 1);
    const int i0 = ((b - j) << 1) + j, i1 = i0 + h;
    const int k = j * (L / h);                      // exp(-i pi j / h) = exp(-i pi k / L)
    const double wr = tw[2 * k], wi = -tw[2 * k + 1];
    const double2 a = z[i0], c = z[i1];
    const double cr = c.x * wr - c.y * wi, ci = c.x * wi + c.y * wr;
    z[i0] = double2{a.x + cr, a.y + ci};
    z[i1] = double2{a.x - cr, a.y - ci};
    __syncthreads();
  }
}

template <int L>
__device__ __forceinline__ int bitrev(int j) {
  return (int)(__brev((unsigned)j) >> (32 - FftBits<L>::value));
}

// Load the odd extensions of two length-m vectors (x1[j - 1], x2[j - 1] read
// through `get`) in bit-reversed order: thread t places entries t and t + L.
// `also` runs after the stores and before the barrier (LDS stores of values
// the caller loaded earlier, so that their loads overlap with these).
template <int L, class Get, class Also>
__device__ __forceinline__ void fst_load(double2* z, int m, Get get, Also also) {
  const int t = threadIdx.x;
  double2 v = double2{0.0, 0.0}, w = double2{0.0, 0.0};
  if (t >= 1 && t <= m) v = get(t - 1);                         // z_t = x_t
  if (t >= 1 && L - t <= m) {                                    // z_{L+t} = -x_{L-t}
    const double2 u = get(L - t - 1);
    w = double2{-u.x, -u.y};
  }
  z[bitrev<L>(t)] = v;
  z[bitrev<L>(t + L)] = w;
  also();
  __syncthreads();
}

template <int L, class Get>
__device__ __forceinline__ void fst_load(double2* z, int m, Get get) {
  fst_load<L>(z, m, get, [] {});
}

}  // namespace sts
