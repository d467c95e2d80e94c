// Direct Mx solves for the 3-D trilinear mass matrix.
//
// The consistent trilinear (Q1) mass matrix on the uniform grid (this
// library's reading of the 3-D discretisation; the paper's 3-D heat problem,
// Sec. 5, Example 1, uses linear elements) is the tensor product of
// three 1-D mass matrices, Mx = (h/6)^3 T (x) T (x) T with T = tridiag(1, 4, 1),
// so Mx^{-1} = (6/h)^3 T^{-1} (x) T^{-1} (x) T^{-1}: three passes, each solving
// T y = x along every grid line of one direction (elimination without
// pivoting; T is strictly diagonally dominant).  The elimination factors of T
// depend only on the line length and are computed once per problem.  One
// thread per line; lines along y and z are read and written coalesced across
// threads, lines along x are staged through LDS in chunks.
#include <hip/hip_runtime.h>

#include "sts_internal.h"

namespace sts {

namespace {

// fac: c (n) | m (n) of T = tridiag(1, 4, 1): m_0 = 1/4, m_i = 1 / (4 - c_{i-1}), c_i = m_i.
__global__ void tensor_factor_kernel(int n, double* fac) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double cp = 0.0;
  for (int i = 0; i < n; ++i) {
    const double mi = 1.0 / (4.0 - cp);
    cp = mi;
    fac[i] = cp;
    fac[n + i] = mi;
  }
}

struct TensorArgs {
  int n;
  int axis;              // 0: x, 1: y, 2: z
  int ncols;
  const double* in[kMaxCols];
  double* out[kMaxCols];
  const double* fac;
  double scale;          // 6 / h, applied once per pass
};

constexpr int kLine = 8;
__global__ __launch_bounds__(256) void tensor_mass_kernel(TensorArgs a) {
  const int n = a.n;
  const int64_t lines = (int64_t)n * n;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (gid >= lines || c >= a.ncols) return;
  int64_t base, stride;
  if (a.axis == 0) {
    base = gid * n;
    stride = 1;
  } else if (a.axis == 1) {
    const int64_t z = gid / n, x = gid % n;
    base = z * n * n + x;
    stride = n;
  } else {
    base = gid;
    stride = lines;
  }
  const double* in = a.in[c] + base;
  double* out = a.out[c] + base;
  const double* cf = a.fac;
  const double* mf = a.fac + n;
  // The recurrences are serial but their loads are not: each chunk of
  // kLine elements is loaded into registers before its steps run, so a
  // thread has kLine loads in flight instead of one.  (In place, in == out:
  // every element is read before the same thread writes it.)
  double y = 0.0;
  for (int i0 = 0; i0 < n; i0 += kLine) {
    double v[kLine], m[kLine];
#pragma unroll
    for (int u = 0; u < kLine; ++u) {
      v[u] = in[min(i0 + u, n - 1) * stride];
      m[u] = mf[min(i0 + u, n - 1)];
    }
#pragma unroll
    for (int u = 0; u < kLine; ++u) {
      const int i = i0 + u;
      if (i < n) {
        y = (a.scale * v[u] - y) * m[u];
        out[i * stride] = y;
      }
    }
  }
  double z = 0.0;
  for (int i1 = n - 1; i1 >= 0; i1 -= kLine) {
    double v[kLine], f[kLine];
#pragma unroll
    for (int u = 0; u < kLine; ++u) {
      v[u] = out[max(i1 - u, 0) * stride];
      f[u] = cf[max(i1 - u, 0)];
    }
#pragma unroll
    for (int u = 0; u < kLine; ++u) {
      const int i = i1 - u;
      if (i >= 0) {
        z = v[u] - f[u] * z;
        out[i * stride] = z;
      }
    }
  }
}

// Lines along x are contiguous, so one thread per line would read 64
// different cache lines per wave access.  Here each wave stages chunks of
// kChunk elements of its 64 lines through LDS: loads and stores are
// coalesced along x, and each thread runs the recurrences of its own line on
// the staged chunk.  Forward sweep left to right (y written out), then the
// backward sweep right to left over y.
constexpr int kChunk = 16;

// Elements x0 .. x0 + kChunk - 1 of the wave's 64 lines into T (zero past the
// grid): branch-free loads (outside, the column's first element is read and
// dropped), all kChunk of a lane issued before the first LDS store.
__device__ __forceinline__ void stage_chunk(double (*T)[kChunk + 1], const double* g, int64_t line0,
                                            int64_t lines, int n, int x0, int lane) {
  double v[kChunk];
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    const int e = lane + 64 * k;
    const int l = e / kChunk, x = e % kChunk;
    const int64_t line = line0 + l;
    const bool in = line < lines && x0 + x < n;
    const double w = g[in ? line * n + x0 + x : 0];
    v[k] = in ? w : 0.0;
  }
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    const int e = lane + 64 * k;
    T[e / kChunk][e % kChunk] = v[k];
  }
}

__global__ __launch_bounds__(256) void tensor_mass_x_kernel(TensorArgs a) {
  __shared__ double tile[4][64][kChunk + 1];
  const int n = a.n;
  const int64_t lines = (int64_t)n * n;
  const int c = blockIdx.y;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t line0 = (int64_t)blockIdx.x * 256 + wv * 64;   // this wave's first line
  const double* in = a.in[c];
  double* out = a.out[c];
  const double* cf = a.fac;
  const double* mf = a.fac + n;
  double (*T)[kChunk + 1] = tile[wv];
  const int nch = (n + kChunk - 1) / kChunk;
  double y = 0.0;
  for (int ch = 0; ch < nch; ++ch) {
    const int x0 = ch * kChunk;
    stage_chunk(T, in, line0, lines, n, x0, lane);
    double m[kChunk];
#pragma unroll
    for (int x = 0; x < kChunk; ++x) m[x] = mf[min(x0 + x, n - 1)];
    __syncthreads();
#pragma unroll
    for (int x = 0; x < kChunk; ++x) {
      if (x0 + x < n) {
        y = (a.scale * T[lane][x] - y) * m[x];
        T[lane][x] = y;
      }
    }
    __syncthreads();
    for (int e = lane; e < 64 * kChunk; e += 64) {
      const int l = e / kChunk, x = e % kChunk;
      const int64_t line = line0 + l;
      if (line < lines && x0 + x < n) out[line * n + x0 + x] = T[l][x];
    }
    __syncthreads();
  }
  double z = 0.0;
  for (int ch = nch - 1; ch >= 0; --ch) {
    const int x0 = ch * kChunk;
    stage_chunk(T, out, line0, lines, n, x0, lane);
    double f[kChunk];
#pragma unroll
    for (int x = 0; x < kChunk; ++x) f[x] = cf[min(x0 + x, n - 1)];
    __syncthreads();
#pragma unroll
    for (int x = kChunk - 1; x >= 0; --x) {
      if (x0 + x < n) {
        z = T[lane][x] - f[x] * z;
        T[lane][x] = z;
      }
    }
    __syncthreads();
    for (int e = lane; e < 64 * kChunk; e += 64) {
      const int l = e / kChunk, x = e % kChunk;
      const int64_t line = line0 + l;
      if (line < lines && x0 + x < n) out[line * n + x0 + x] = T[l][x];
    }
    __syncthreads();
  }
}

}  // namespace

bool tensor_mass_supported(const Grid& g, const Stencil& M) {
  if (g.dim != 3 || g.nx != g.ny || g.nx != g.nz) return false;
  const double s = M.c[13] / 64.0;   // centre = s 4^3
  if (!(s > 0.0)) return false;
  const double w[3] = {1.0, 4.0, 1.0};
  for (int dz = 0; dz < 3; ++dz)
    for (int dy = 0; dy < 3; ++dy)
      for (int dx = 0; dx < 3; ++dx) {
        const double want = s * w[dx] * w[dy] * w[dz];
        const double got = M.c[(dz * 3 + dy) * 3 + dx];
        if (std::fabs(got - want) > 1e-14 * s * 64.0) return false;
      }
  return true;
}

void tensor_mass_factor(int n, double* fac, hipStream_t st) {
  tensor_factor_kernel<<<1, 64, 0, st>>>(n, fac);
  STS_HIP(hipGetLastError());
}

void tensor_mass_solve(const Grid& g, const Stencil& M, int ncols, const double* const* b,
                       double* x, int64_t ldx, const double* fac, hipStream_t st) {
  STS_REQUIRE(ncols >= 0 && ncols <= kMaxCols, STS_E_INVALID, "tensor mass solve: 0..8 columns");
  if (ncols == 0) return;
  const int n = g.nx;
  // Mx = s (4^3) ... with s = (h/6)^3: the per-pass factor is s^{-1/3} = 6 / h
  const double s = M.c[13] / 64.0;
  TensorArgs a{};
  a.n = n;
  a.ncols = ncols;
  a.fac = fac;
  a.scale = 1.0 / std::cbrt(s);
  const int64_t lines = (int64_t)n * n;
  const dim3 grid((unsigned)((lines + 255) / 256), (unsigned)ncols);
  for (int axis = 0; axis < 3; ++axis) {
    a.axis = axis;
    for (int c = 0; c < ncols; ++c) {
      a.in[c] = axis == 0 ? b[c] : x + c * ldx;
      a.out[c] = x + c * ldx;
    }
    // read and write every node once per pass (the x pass twice: y is stored
    // between its sweeps)
    if (axis == 0)
      launch(STS_K_MASS_CHEB, 32.0 * (double)g.nh * ncols, tensor_mass_x_kernel, grid, dim3(256),
             0, st, a);
    else
      launch(STS_K_MASS_CHEB, 16.0 * (double)g.nh * ncols, tensor_mass_kernel, grid, dim3(256), 0,
             st, a);
    STS_HIP(hipGetLastError());
  }
}

}  // namespace sts
