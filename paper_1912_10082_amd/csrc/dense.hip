// Dense kernels of the projection step, FP64 on the CDNA4 matrix cores.
//
// The block Gram-Schmidt of the extended Krylov basis contracts the tall
// basis V (Nh x k) with a thin block W (Nh x <= 16): C = V^T W and W -= V C.
// Both are HBM-bound (about one flop per byte); the matrix cores are used
// for the contraction itself through v_mfma_f64_16x16x4f64.  With lane
// l = i + 16 g supplying a = X[i][g] and b = Y[g][i], element q of lane l's
// accumulator is (X Y)[4 q + g][i] (measured on gfx950: columns of the product
// follow the lane within a 16-lane group, rows follow the group and the
// accumulator element).
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>

#include "sts_internal.h"

namespace sts {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Work split of C = A^T B: a work-group takes T consecutive 16-column tiles
// of A (one accumulator each, so a wave runs T independent MFMA chains and
// loads each B value once for all of them) over NW * rpw consecutive rows,
// NW waves taking rpw rows each.  At most kMaxChunks row chunks keep the
// cross-chunk reduction to a few loads per lane.
constexpr int kMaxChunks = 256;

struct TnPlan {
  int T, NW, rpw;
  int64_t nch;
  int groups;
};

// nw > 0 overrides the waves per work-group of the chosen tile count
TnPlan tn_plan(int64_t rows, int m, int nw = 0) {
  TnPlan p{};
  const int tiles = (m + 15) / 16;
  // four tiles per work-group once there are at least two such groups; below
  // that two tiles, so that narrow bases still spread over two or more groups
  // (m = 60 on 261121 rows: 4.0 TB/s against 2.9 TB/s with one 4-tile group)
  p.T = tiles >= 8 ? 4 : (tiles >= 2 ? 2 : 1);
  p.NW = nw > 0 ? nw : (p.T == 1 ? 16 : 4);
  p.groups = (tiles + p.T - 1) / p.T;
  // about 512 work-groups in all, at least 64 rows per wave
  const int64_t target = std::max<int64_t>(1, std::min<int64_t>(kMaxChunks, 512 / p.groups));
  const int64_t per = (std::max<int64_t>(rows, 1) + p.NW * target - 1) / (p.NW * target);
  p.rpw = (int)std::max<int64_t>(64, (per + 15) / 16 * 16);
  p.nch = std::max<int64_t>(1, (rows + (int64_t)p.NW * p.rpw - 1) / ((int64_t)p.NW * p.rpw));
  return p;
}

// partial[chunk][c][j] (c < m16, j < 16) of A^T B over the chunk's rows.
// Columns j < n1 of B come from B1, the rest from B2 (same leading dimension).
// Lane (i, g) of a wave feeds rows r + 4 g .. r + 4 g + 3 of column i of each
// tile to the four MFMAs of a 16-row step; VEC reads them as two 16-byte
// loads (columns 16-byte aligned, even leading dimensions).
template <int T, int NW, bool VEC>
__global__ __launch_bounds__(64 * NW) void gemm_tn_kernel(int64_t rows, int m, int n,
                                                          const double* A, int64_t lda,
                                                          const double* B1, const double* B2,
                                                          int n1, int64_t ldb, double* partial,
                                                          int m16, int rpw) {
  __shared__ double red[NW - 1][T][256];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int c0 = blockIdx.x * 16 * T;
  const int64_t chunk = blockIdx.y;
  const int64_t rb = (chunk * NW + wv) * (int64_t)rpw;
  const int64_t re = min(rb + rpw, rows);
  const double* Ap[T];
  bool aok[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int col = c0 + 16 * t + i;
    aok[t] = col < m;
    Ap[t] = A + (int64_t)(aok[t] ? col : 0) * lda;
  }
  const bool bok = i < n;
  const double* Bp = !bok ? B1 : (i < n1 ? B1 + (int64_t)i * ldb : B2 + (int64_t)(i - n1) * ldb);
  d4 acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  int64_t r = rb;
  for (; r + 16 <= re; r += 16) {
    const int64_t rr = r + 4 * g;
    double av[T][4], bv[4];
    if (VEC) {
      const double2 b0 = bok ? *(const double2*)(Bp + rr) : double2{0.0, 0.0};
      const double2 b1 = bok ? *(const double2*)(Bp + rr + 2) : double2{0.0, 0.0};
      bv[0] = b0.x;
      bv[1] = b0.y;
      bv[2] = b1.x;
      bv[3] = b1.y;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const double2 a0 = aok[t] ? *(const double2*)(Ap[t] + rr) : double2{0.0, 0.0};
        const double2 a1 = aok[t] ? *(const double2*)(Ap[t] + rr + 2) : double2{0.0, 0.0};
        av[t][0] = a0.x;
        av[t][1] = a0.y;
        av[t][2] = a1.x;
        av[t][3] = a1.y;
      }
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        bv[s] = bok ? Bp[rr + s] : 0.0;
#pragma unroll
        for (int t = 0; t < T; ++t) av[t][s] = aok[t] ? Ap[t][rr + s] : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < T; ++t) acc[t] = mfma(av[t][s], bv[s], acc[t]);
  }
  if (r < re) {   // ragged end of the wave's rows
    const int64_t rr = r + 4 * g;
    double av[T][4], bv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool ok = rr + s < re;
      bv[s] = (ok && bok) ? Bp[rr + s] : 0.0;
#pragma unroll
      for (int t = 0; t < T; ++t) av[t][s] = (ok && aok[t]) ? Ap[t][rr + s] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < T; ++t) acc[t] = mfma(av[t][s], bv[s], acc[t]);
  }
  // element q of a lane's accumulator is (tile row 4 q + g, column i)
  if (wv > 0) {
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[wv - 1][t][(4 * q + g) * 16 + i] = acc[t][q];
  }
  __syncthreads();
  if (wv != 0) return;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    if (c0 + 16 * t >= m16) break;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = (4 * q + g) * 16 + i;
      double v = acc[t][q];
#pragma unroll
      for (int w = 0; w < NW - 1; ++w) v += red[w][t][e];
      partial[(chunk * m16 + c0 + 16 * t + 4 * q + g) * 16 + i] = v;
    }
  }
}

// One wave per output element: lanes take chunks lane, lane + 64, ... and the
// lane sums are combined in a fixed order.  Columns j < n1 go to C1, the rest
// to C2.
__global__ __launch_bounds__(256) void gemm_tn_reduce(int m, int n, int64_t nchunks, int m16,
                                                      const double* partial, double* C1,
                                                      double* C2, int n1, int64_t ldc) {
  const int idx = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (idx >= m * n) return;
  const int i = idx % m, j = idx / m;
  double s = 0.0;
  // unrolled so that eight loads are in flight per trip (same summation order)
#pragma unroll 8
  for (int64_t c = lane; c < nchunks; c += 64) s += partial[(c * m16 + i) * 16 + j];
  s = wave_sum(s);
  if (lane == 0) {
    if (j < n1) C1[i + (int64_t)j * ldc] = s;
    else C2[i + (int64_t)(j - n1) * ldc] = s;
  }
}

// ---------------------------------------------------------------------------
// FP32 form of the Gram-Schmidt contraction (the coefficients of the first
// classical Gram-Schmidt pass of the mixed-precision solve): A is an FP32
// copy of the basis, the thin FP64 operand is rounded to FP32 as it is
// loaded, products and sums are FP32 on v_mfma_f32_16x16x4f32.  Its operands are laid out as
// in the FP64 16x16x4 instruction above (lane i + 16 g supplies a = X[i][g],
// b = Y[g][i]), but its accumulator is not: element q of lane i + 16 g is
// (X Y)[4 g + q][i] (four consecutive rows per lane group).
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float wave_sum32(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// partial[chunk][c][j] (c < m16, j < 16) of A^T B over the chunk's rows, in
// FP32; the work split of gemm_tn_kernel.  VEC: one 16-byte load of four A
// rows and two of four B rows per lane (A 16-byte aligned with ld % 4 == 0,
// B 16-byte aligned with even ld).
template <int T, int NW, bool VEC>
__global__ __launch_bounds__(64 * NW) void gemm_tn32_kernel(int64_t rows, int m, int n,
                                                            const float* A, int64_t lda,
                                                            const double* B, int64_t ldb,
                                                            float* partial, int m16, int rpw) {
  __shared__ float red[NW - 1][T][256];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int c0 = blockIdx.x * 16 * T;
  const int64_t chunk = blockIdx.y;
  const int64_t rb = (chunk * NW + wv) * (int64_t)rpw;
  const int64_t re = min(rb + rpw, rows);
  const float* Ap[T];
  bool aok[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int col = c0 + 16 * t + i;
    aok[t] = col < m;
    Ap[t] = A + (int64_t)(aok[t] ? col : 0) * lda;
  }
  const bool bok = i < n;
  const double* Bp = B + (int64_t)(bok ? i : 0) * ldb;
  f4 acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  int64_t r = rb;
  if (VEC) {
    // 32 rows per step: lane group g feeds rows r + 8 g .. r + 8 g + 7 (two
    // 16-byte loads of A per tile, as many bytes in flight as the FP64
    // kernel's 16-row step) to eight MFMAs
    for (; r + 32 <= re; r += 32) {
      const int64_t rr = r + 8 * g;
      float av[T][8], bv[8];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const double2 b2 = bok ? *(const double2*)(Bp + rr + 2 * h) : double2{0.0, 0.0};
        bv[2 * h] = (float)b2.x;
        bv[2 * h + 1] = (float)b2.y;
      }
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const float4 a0 = aok[t] ? *(const float4*)(Ap[t] + rr) : float4{0.0f, 0.0f, 0.0f, 0.0f};
        const float4 a1 =
            aok[t] ? *(const float4*)(Ap[t] + rr + 4) : float4{0.0f, 0.0f, 0.0f, 0.0f};
        av[t][0] = a0.x;
        av[t][1] = a0.y;
        av[t][2] = a0.z;
        av[t][3] = a0.w;
        av[t][4] = a1.x;
        av[t][5] = a1.y;
        av[t][6] = a1.z;
        av[t][7] = a1.w;
      }
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int t = 0; t < T; ++t) acc[t] = mfma32(av[t][s], bv[s], acc[t]);
    }
  }
  for (; r + 16 <= re; r += 16) {
    const int64_t rr = r + 4 * g;
    float av[T][4], bv[4];
    if (VEC) {
      const double2 b0 = bok ? *(const double2*)(Bp + rr) : double2{0.0, 0.0};
      const double2 b1 = bok ? *(const double2*)(Bp + rr + 2) : double2{0.0, 0.0};
      bv[0] = (float)b0.x;
      bv[1] = (float)b0.y;
      bv[2] = (float)b1.x;
      bv[3] = (float)b1.y;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const float4 a4 = aok[t] ? *(const float4*)(Ap[t] + rr) : float4{0.0f, 0.0f, 0.0f, 0.0f};
        av[t][0] = a4.x;
        av[t][1] = a4.y;
        av[t][2] = a4.z;
        av[t][3] = a4.w;
      }
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        bv[s] = bok ? (float)Bp[rr + s] : 0.0f;
#pragma unroll
        for (int t = 0; t < T; ++t) av[t][s] = aok[t] ? Ap[t][rr + s] : 0.0f;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < T; ++t) acc[t] = mfma32(av[t][s], bv[s], acc[t]);
  }
  if (r < re) {   // ragged end of the wave's rows
    const int64_t rr = r + 4 * g;
    float av[T][4], bv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool ok = rr + s < re;
      bv[s] = (ok && bok) ? (float)Bp[rr + s] : 0.0f;
#pragma unroll
      for (int t = 0; t < T; ++t) av[t][s] = (ok && aok[t]) ? Ap[t][rr + s] : 0.0f;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < T; ++t) acc[t] = mfma32(av[t][s], bv[s], acc[t]);
  }
  // element q of a lane's accumulator is (tile row 4 g + q, column i)
  if (wv > 0) {
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[wv - 1][t][(4 * g + q) * 16 + i] = acc[t][q];
  }
  __syncthreads();
  if (wv != 0) return;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    if (c0 + 16 * t >= m16) break;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = (4 * g + q) * 16 + i;
      float v = acc[t][q];
#pragma unroll
      for (int w = 0; w < NW - 1; ++w) v += red[w][t][e];
      partial[(chunk * m16 + c0 + 16 * t + 4 * g + q) * 16 + i] = v;
    }
  }
}

// C (m x n, FP64 storage) = the sum of the FP32 chunk partials, in FP32.
__global__ __launch_bounds__(256) void gemm_tn32_reduce(int m, int n, int64_t nchunks, int m16,
                                                        const float* partial, double* C,
                                                        int64_t ldc) {
  const int idx = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (idx >= m * n) return;
  const int i = idx % m, j = idx / m;
  float s = 0.0f;
  for (int64_t c = lane; c < nchunks; c += 64) s += partial[(c * m16 + i) * 16 + j];
  s = wave_sum32(s);
  if (lane == 0) C[i + (int64_t)j * ldc] = (double)s;
}

// FP64 -> FP32 copy of columns (the FP32 copy of new basis columns).
__global__ void round_cols_kernel(int64_t rows, int ncols, const double* src, int64_t lds,
                                  float* dst, int64_t ldd) {
  for (int c = blockIdx.y; c < ncols; c += gridDim.y)
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * blockDim.x)
      dst[r + (int64_t)c * ldd] = (float)src[r + (int64_t)c * lds];
}

// The contraction with up to 32 columns of B in up to three segments (each
// with its own pointer, common ldb): NB 16-column tiles of B per wave, the
// work split of gemm_tn_kernel.  The Gram-Schmidt pass that re-orthogonalises
// a new block contracts the basis with the block and, in the same read, with
// the Kx / Mx images of the previous block (its reduced-matrix columns).
struct TnSegs {
  const double* B[3];
  int end[3];   // cumulative column counts: segment s holds columns [end[s-1], end[s])
};

__device__ __forceinline__ const double* seg_col(const TnSegs& s, int j, int64_t ldb) {
  const int g = j < s.end[0] ? 0 : (j < s.end[1] ? 1 : 2);
  const int j0 = g == 0 ? 0 : s.end[g - 1];
  return s.B[g] + (int64_t)(j - j0) * ldb;
}

template <int T, int NW, int NB, bool VEC>
__global__ __launch_bounds__(64 * NW) void gemm_tnw_kernel(int64_t rows, int m, int n,
                                                           const double* A, int64_t lda,
                                                           TnSegs segs, int64_t ldb,
                                                           double* partial, int m16, int rpw) {
  __shared__ double red[NW - 1][T][NB][256];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int c0 = blockIdx.x * 16 * T;
  const int64_t chunk = blockIdx.y;
  const int64_t rb = (chunk * NW + wv) * (int64_t)rpw;
  const int64_t re = min(rb + rpw, rows);
  const double* Ap[T];
  bool aok[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int col = c0 + 16 * t + i;
    aok[t] = col < m;
    Ap[t] = A + (int64_t)(aok[t] ? col : 0) * lda;
  }
  const double* Bp[NB];
  bool bok[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int j = 16 * u + i;
    bok[u] = j < n;
    Bp[u] = seg_col(segs, bok[u] ? j : 0, ldb);
  }
  d4 acc[T][NB];
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int u = 0; u < NB; ++u) acc[t][u] = d4{0.0, 0.0, 0.0, 0.0};
  int64_t r = rb;
  for (; r + 16 <= re; r += 16) {
    const int64_t rr = r + 4 * g;
    double av[T][4], bv[NB][4];
    if (VEC) {
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const double2 b0 = bok[u] ? *(const double2*)(Bp[u] + rr) : double2{0.0, 0.0};
        const double2 b1 = bok[u] ? *(const double2*)(Bp[u] + rr + 2) : double2{0.0, 0.0};
        bv[u][0] = b0.x;
        bv[u][1] = b0.y;
        bv[u][2] = b1.x;
        bv[u][3] = b1.y;
      }
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const double2 a0 = aok[t] ? *(const double2*)(Ap[t] + rr) : double2{0.0, 0.0};
        const double2 a1 = aok[t] ? *(const double2*)(Ap[t] + rr + 2) : double2{0.0, 0.0};
        av[t][0] = a0.x;
        av[t][1] = a0.y;
        av[t][2] = a1.x;
        av[t][3] = a1.y;
      }
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int u = 0; u < NB; ++u) bv[u][s] = bok[u] ? Bp[u][rr + s] : 0.0;
#pragma unroll
        for (int t = 0; t < T; ++t) av[t][s] = aok[t] ? Ap[t][rr + s] : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int u = 0; u < NB; ++u) acc[t][u] = mfma(av[t][s], bv[u][s], acc[t][u]);
  }
  if (r < re) {   // ragged end of the wave's rows
    const int64_t rr = r + 4 * g;
    double av[T][4], bv[NB][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool ok = rr + s < re;
#pragma unroll
      for (int u = 0; u < NB; ++u) bv[u][s] = (ok && bok[u]) ? Bp[u][rr + s] : 0.0;
#pragma unroll
      for (int t = 0; t < T; ++t) av[t][s] = (ok && aok[t]) ? Ap[t][rr + s] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int u = 0; u < NB; ++u) acc[t][u] = mfma(av[t][s], bv[u][s], acc[t][u]);
  }
  // element q of a lane's accumulator is (tile row 4 q + g, column i)
  if (wv > 0) {
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int u = 0; u < NB; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) red[wv - 1][t][u][(4 * q + g) * 16 + i] = acc[t][u][q];
  }
  __syncthreads();
  if (wv != 0) return;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    if (c0 + 16 * t >= m16) break;
#pragma unroll
    for (int u = 0; u < NB; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = (4 * q + g) * 16 + i;
        double v = acc[t][u][q];
#pragma unroll
        for (int w = 0; w < NW - 1; ++w) v += red[w][t][u][e];
        partial[(chunk * m16 + c0 + 16 * t + 4 * q + g) * (16 * NB) + 16 * u + i] = v;
      }
  }
}

struct TnOut {
  double* C[3];
  int64_t ldc[3];
  int end[3];
};

// One wave per output element, chunks summed in a fixed order; column j goes
// to the output segment that holds it.
__global__ __launch_bounds__(256) void gemm_tnw_reduce(int m, int n, int64_t nchunks, int m16,
                                                       int width, const double* partial,
                                                       TnOut out) {
  const int idx = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (idx >= m * n) return;
  const int i = idx % m, j = idx / m;
  double s = 0.0;
  // unrolled so that eight loads are in flight per trip (same summation order)
#pragma unroll 8
  for (int64_t c = lane; c < nchunks; c += 64) s += partial[(c * m16 + i) * width + j];
  s = wave_sum(s);
  if (lane == 0) {
    const int g = j < out.end[0] ? 0 : (j < out.end[1] ? 1 : 2);
    const int j0 = g == 0 ? 0 : out.end[g - 1];
    out.C[g][i + (int64_t)(j - j0) * out.ldc[g]] = s;
  }
}

// W (rows x n) -= A (rows x m) C (m x n); each wave owns 16 rows.
__global__ __launch_bounds__(256) void gemm_nn_sub_kernel(int64_t rows, int m, int n,
                                                          const double* A, int64_t lda,
                                                          const double* C, int64_t ldc, double* W,
                                                          int64_t ldw) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + wv) * 16;
  if (r0 >= rows) return;
  const bool rok = (r0 + i) < rows;
  const bool cok = i < n;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < m; k0 += 4) {
    const int kk = k0 + g;
    const double a = (rok && kk < m) ? A[(r0 + i) + (int64_t)kk * lda] : 0.0;
    const double b = (cok && kk < m) ? C[kk + (int64_t)i * ldc] : 0.0;
    acc = mfma(a, b, acc);
  }
  if (cok) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = r0 + 4 * q + g;
      if (row < rows) W[row + (int64_t)i * ldw] -= acc[q];
    }
  }
}

// The same product with 64 rows per wave: lane (i, g) feeds rows
// r0 + 4 i .. r0 + 4 i + 3 of column k0 + g to four MFMAs with independent
// accumulators (one 32-byte load per lane and step, four chains instead of
// one); accumulator s of the lane holds rows r0 + 4 (4 q + g) + s.
template <bool VEC>
__global__ __launch_bounds__(256) void gemm_nn_sub4_kernel(int64_t rows, int m, int n,
                                                           const double* A, int64_t lda,
                                                           const double* C, int64_t ldc,
                                                           double* W, int64_t ldw) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + wv) * 64;
  if (r0 >= rows) return;
  const int64_t ra = r0 + 4 * i;
  const bool cok = i < n;
  d4 acc[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) acc[s] = d4{0.0, 0.0, 0.0, 0.0};
  // Two copies of the k loop: 32-byte loads for waves whose 64 rows all
  // exist, guarded scalar loads for the last one.  Every load is
  // branch-free (ap and the C index stay in bounds past m), so a step's
  // loads are in flight together.
  auto k_loop = [&](auto wide) {
    for (int k0 = 0; k0 < m; k0 += 4) {
      const int kk = k0 + g;
      const bool kok = kk < m;
      const double* ap = A + ra + (int64_t)(kok ? kk : 0) * lda;
      const double c = C[(kok ? kk : 0) + (int64_t)(cok ? i : 0) * ldc];
      double a[4];
      if constexpr (decltype(wide)::value) {
        const double2 x = *(const double2*)ap;
        const double2 y = *(const double2*)(ap + 2);
        a[0] = kok ? x.x : 0.0;
        a[1] = kok ? x.y : 0.0;
        a[2] = kok ? y.x : 0.0;
        a[3] = kok ? y.y : 0.0;
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) a[s] = (kok && ra + s < rows) ? ap[s] : 0.0;
      }
      const double b = (cok && kok) ? c : 0.0;
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[s] = mfma(a[s], b, acc[s]);
    }
  };
  if (VEC && r0 + 63 < rows)
    k_loop(std::true_type{});
  else
    k_loop(std::false_type{});
  if (cok) {
    // the old values of the lane's outputs, four in flight together (rows
    // past the end read row r0 and are not written back; four at a time
    // keeps the register count, and so the occupancy, of the main loop)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double w[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t row = r0 + 4 * (4 * q + g) + s;
        w[s] = W[(row < rows ? row : r0) + (int64_t)i * ldw];
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t row = r0 + 4 * (4 * q + g) + s;
        if (row < rows) W[row + (int64_t)i * ldw] = w[s] - acc[s][q];
      }
    }
  }
}

// D (m x n) = A (m x kk) B (kk x n); each wave one 16x16 tile.
// D = alpha op(A) B + beta D with op(A) = A (m x kk) or A^T (A: kk x m); one
// wave per 16 x 16 tile of D.
template <bool TA>
__global__ __launch_bounds__(256) void gemm_small_kernel(int m, int n, int kk, double alpha,
                                                         const double* A, int64_t lda,
                                                         const double* B, int64_t ldb,
                                                         double beta, double* D, int64_t ldd) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int tiles_m = (m + 15) / 16;
  const int tile = blockIdx.x * 4 + wv;
  const int tm = tile % tiles_m, tn = tile / tiles_m;
  if (tn * 16 >= n) return;
  const int r0 = tm * 16, c0 = tn * 16;
  const bool rok = (r0 + i) < m;
  const bool cok = (c0 + i) < n;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < kk; k0 += 4) {
    const int k = k0 + g;
    double a = 0.0;
    if (rok && k < kk) a = TA ? A[k + (int64_t)(r0 + i) * lda] : A[(r0 + i) + (int64_t)k * lda];
    const double b = (cok && k < kk) ? B[k + (int64_t)(c0 + i) * ldb] : 0.0;
    acc = mfma(a, b, acc);
  }
  if (cok) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = r0 + 4 * q + g;
      if (row < m) {
        double* d = D + row + (int64_t)(c0 + i) * ldd;
        *d = beta == 0.0 ? alpha * acc[q] : alpha * acc[q] + beta * *d;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// || [A_0 A_1 A_2] B ||_F^2 with B given transposed (BT: n x mtot).
// Work-group tile: 64 rows x 256 columns; wave w owns columns [64 w, 64 w + 64)
// as 4 x 4 independent 16 x 16 MFMA accumulators.  Each segment A_s is swept
// on its own (its k-steps never straddle two segments) with the operands of
// the next kPD k-steps in flight (three slots measured 17% faster than
// loading one step ahead: 5.2 against 6.3 ms for 261121 x 442 x 1024).
// ---------------------------------------------------------------------------
constexpr int kPD = 3;

struct ResArgs {
  int64_t rows;
  int n;
  int nseg;
  const double* A[3];
  int64_t lda[3];
  int m[3];
  const double* BT;
  int64_t ldbt;
  int upper;        // 1: BT[j][t] = 0 for j < t (a triangular factor), rows j < t skipped
  double* partial;
  unsigned* counter;
  double* out;
};

// VEC: row tiles 0 / 1 take the even / odd rows of r0 .. r0 + 31 and tiles
// 2 / 3 those of r0 + 32 .. r0 + 63, so one 16-byte load feeds two tiles
// (segments 16-byte aligned with even leading dimensions).  The sum of
// squares does not depend on which rows a tile holds.
// Two work-groups per CU (the register budget this allows keeps all sixteen
// accumulators and the prefetched operands resident) measured 1.4x faster
// than the compiler's default budget.
template <bool VEC>
__global__ __launch_bounds__(256, 2) void residual_kernel(ResArgs a) {
  __shared__ double red[4];
  __shared__ int last;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 256 + wv * 64;
  const bool full = r0 + 64 <= a.rows;
  d4 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
  int kb = 0;   // first row of BT of the segment
  // with a triangular BT this wave's columns c0 .. c0 + 63 need rows j >= c0
  const int kfirst = a.upper ? (c0 & ~3) : 0;
  for (int s = 0; s < a.nseg; ++s) {
    const double* A = a.A[s];
    const int64_t lda = a.lda[s];
    const int m = a.m[s];
    const int k00 = kfirst > kb ? ((kfirst - kb) & ~3) : 0;
    if (k00 >= m) {
      kb += m;
      continue;
    }
    auto load = [&](int k0, double* av, double* bv) {
      const int kk = k0 + g;
      const bool kok = kk < m;
      const double* bt = a.BT + (int64_t)(kb + (kok ? kk : 0)) * a.ldbt;
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        const int col = c0 + 16 * y + i;
        bv[y] = (kok && col < a.n) ? bt[col] : 0.0;
      }
      const double* ap = A + (int64_t)(kok ? kk : 0) * lda;
      if (VEC && full) {
        const double2 lo = kok ? *(const double2*)(ap + r0 + 2 * i) : double2{0.0, 0.0};
        const double2 hi = kok ? *(const double2*)(ap + r0 + 32 + 2 * i) : double2{0.0, 0.0};
        av[0] = lo.x;
        av[1] = lo.y;
        av[2] = hi.x;
        av[3] = hi.y;
      } else {
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const int64_t row = VEC ? r0 + 32 * (x >> 1) + 2 * i + (x & 1) : r0 + 16 * x + i;
          av[x] = (kok && row < a.rows) ? ap[row] : 0.0;
        }
      }
    };
    // kPD operand slots in flight: slot p holds k-step k0 + 4 p and is
    // refilled with the step kPD ahead as soon as its products are issued
    // (loads past the segment's end read zeros)
    double av[kPD][4], bv[kPD][4];
#pragma unroll
    for (int p = 0; p < kPD; ++p) load(k00 + 4 * p, av[p], bv[p]);
    for (int k0 = k00; k0 < m; k0 += 4 * kPD) {
#pragma unroll
      for (int p = 0; p < kPD; ++p) {
        if (k0 + 4 * p < m) {
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] = mfma(av[p][x], bv[p][y], acc[x][y]);
          load(k0 + 4 * (p + kPD), av[p], bv[p]);
        }
      }
    }
    kb += m;
  }
  double s = 0.0;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) s += acc[x][y][q] * acc[x][y][q];
  s = wave_sum(s);
  if (lane == 0) red[wv] = s;
  __syncthreads();
  const int nblk = gridDim.x * gridDim.y;
  const int bid = blockIdx.x + gridDim.x * blockIdx.y;
  if (threadIdx.x == 0) {
    a.partial[bid] = (red[0] + red[1]) + (red[2] + red[3]);
    __threadfence();
    const unsigned prev = atomicAdd(a.counter, 1u);
    last = prev == (unsigned)(nblk - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double t = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) t += a.partial[b];
  t = wave_sum(t);
  __syncthreads();
  if (lane == 0) red[wv] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    *a.out = (red[0] + red[1]) + (red[2] + red[3]);
    atomicExch(a.counter, 0u);
  }
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Cholesky-based column selection on a b x b Gram matrix (one thread).
// A column is dropped if its norm^2 G[c][c] is below defl_v^2 norm0[c] (it was
// already in the span of the basis it was orthogonalised against; G[c][c] is
// a directly computed norm, so this test is accurate to rounding), or if its
// remainder after the earlier kept columns of the block falls below
// defl_b^2 G[c][c] (a Gram-based test, resolvable only to about sqrt(eps)).
// The factorisation runs on one thread with every array in LDS (private
// arrays indexed at run time would live in scratch memory); the columns of
// R^{-1} are then solved in parallel, one thread per column.
__global__ __launch_bounds__(64) void chol_deflate_kernel(int b, const double* G, int64_t ldg,
                                                          const double* norm0, double defl_v,
                                                          double defl_b, double* Rinv,
                                                          CholInfo* info) {
  __shared__ double Gs[16][17];
  __shared__ double L[16][17];
  __shared__ double X[16][17];
  __shared__ double v[16];
  __shared__ int kept_s;
  const int t = threadIdx.x;
  for (int e = t; e < b * b; e += blockDim.x) Gs[e % b][e / b] = G[e % b + (e / b) * ldg];
  __syncthreads();
  if (t == 0) {
    int idx[16];
    int kept = 0;
    double rmin = 1.0;
    for (int c = 0; c < b; ++c) {
      const double gcc = Gs[c][c];
      if (!(gcc == gcc) || !(gcc > 0.0)) continue;
      if (norm0 && !(gcc > defl_v * defl_v * norm0[c])) continue;
      double d = gcc;
      for (int j = 0; j < kept; ++j) {
        double sj = Gs[c][idx[j]];
        for (int q = 0; q < j; ++q) sj -= v[q] * L[j][q];
        v[j] = sj / L[j][j];
        d -= v[j] * v[j];
      }
      if (!(d > defl_b * defl_b * gcc) || !(d == d)) continue;
      rmin = fmin(rmin, sqrt(d / gcc));
      for (int j = 0; j < kept; ++j) L[kept][j] = v[j];
      L[kept][kept] = sqrt(d);
      idx[kept] = c;
      ++kept;
    }
    kept_s = kept;
    info->kept = kept;
    info->rmin = rmin;
    for (int j = 0; j < 16; ++j) info->idx[j] = j < kept ? idx[j] : -1;
    info->ok = 1;
  }
  __syncthreads();
  const int kept = kept_s;
  // R = L^T (upper); thread j solves R x = e_j and writes column j of R^{-1}
  const int j = t;
  if (j < kept) {
    for (int i = kept - 1; i >= 0; --i) {
      double sx = (i == j) ? 1.0 : 0.0;
      for (int q = i + 1; q < kept; ++q) sx -= L[q][i] * X[q][j];
      X[i][j] = sx / L[i][i];
    }
  }
  if (j < b)
    for (int i = 0; i < b; ++i) Rinv[i + j * b] = (j < kept && i <= j) ? X[i][j] : 0.0;
}
__global__ __launch_bounds__(256) void apply_rinv_kernel(int64_t rows, int b, const CholInfo* info,
                                                         const double* Rinv, double* W, double* MW,
                                                         int64_t ldw) {
  // R^-1 (b <= 16) in LDS: every row uses all of it, and read from global
  // memory inside the triangular loop below each product waited on a load
  __shared__ double R[16 * 16];
  if ((int)threadIdx.x < b * b) R[threadIdx.x] = Rinv[threadIdx.x];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int kept = info->kept;
  double w[16], mw[16];
  for (int j = 0; j < kept; ++j) {
    const int c = info->idx[j];
    w[j] = W[r + c * ldw];
    mw[j] = MW ? MW[r + c * ldw] : 0.0;
  }
  for (int j = 0; j < kept; ++j) {
    double s = 0.0, t = 0.0;
    for (int i = 0; i <= j; ++i) {
      const double q = R[i + j * b];
      s += w[i] * q;
      t += mw[i] * q;
    }
    W[r + j * ldw] = s;
    if (MW) MW[r + j * ldw] = t;
  }
}

// Grid-stride over rows (x) and columns (y): any size fits a bounded grid.
__global__ void copy_cols_kernel(int64_t rows, int ncols, const double* src, int64_t lds,
                                 double* dst, int64_t ldd) {
  for (int c = blockIdx.y; c < ncols; c += gridDim.y)
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * blockDim.x)
      dst[r + (int64_t)c * ldd] = src[r + (int64_t)c * lds];
}

__global__ void scale_kernel(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v == 0.0 ? 0.0 : v * p[i];
}

__global__ void fill_kernel(double* p, int64_t n, double v) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x)
    p[idx] = v;
}

__global__ void sumsq_kernel(int64_t rows, int ncols, const double* A, int64_t lda,
                             double* partial, unsigned* counter, double* out) {
  __shared__ double red[4];
  __shared__ int last;
  const int64_t total = rows * ncols;
  double s = 0.0;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * 256) {
    const double v = A[(idx % rows) + (idx / rows) * lda];
    s += v * v;
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
  for (int b = threadIdx.x; b < (int)gridDim.x; b += 256) t += partial[b];
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

int64_t gemm_tn_partial_size(int64_t rows, int m) {
  // every plan has at most min(kMaxChunks, ceil(rows / 256)) chunks
  const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(kMaxChunks, (rows + 255) / 256));
  return nch * (int64_t)(((m + 15) / 16) * 16) * 16;
}

template <int T, int NW>
static void launch_tn(bool vec, const TnPlan& p, int64_t rows, int m, int n, const double* A,
                      int64_t lda, const double* B1, const double* B2, int n1, int64_t ldb,
                      double* partial, int m16, hipStream_t st) {
  const dim3 grid((unsigned)p.groups, (unsigned)p.nch);
  const double bytes = 8.0 * (double)rows * (m + n);
  if (vec)
    launch(STS_K_GRAM, bytes, gemm_tn_kernel<T, NW, true>, grid, dim3(64 * NW), 0, st, rows, m, n,
           A, lda, B1, B2, n1, ldb, partial, m16, p.rpw);
  else
    launch(STS_K_GRAM, bytes, gemm_tn_kernel<T, NW, false>, grid, dim3(64 * NW), 0, st, rows, m,
           n, A, lda, B1, B2, n1, ldb, partial, m16, p.rpw);
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

void gemm_tn2(int64_t rows, int m, int n1, int n2, const double* A, int64_t lda,
              const double* B1, const double* B2, int64_t ldb, double* C1, double* C2,
              int64_t ldc, double* partial, hipStream_t st) {
  const int n = n1 + n2;
  if (m <= 0 || n <= 0) return;
  STS_REQUIRE(n <= 16 && n1 >= 0 && n2 >= 0, STS_E_INVALID, "gemm_tn: n > 16");
  const int m16 = ((m + 15) / 16) * 16;
  const TnPlan p = tn_plan(rows, m);
  if (rows <= 0) {
    fill_kernel<<<1, 256, 0, st>>>(partial, (int64_t)m16 * 16, 0.0);
  } else {
    const bool vec = aligned16(A) && aligned16(B1) && (n2 == 0 || aligned16(B2)) &&
                     lda % 2 == 0 && ldb % 2 == 0;
    if (p.T == 4)
      launch_tn<4, 4>(vec, p, rows, m, n, A, lda, B1, B2, n1, ldb, partial, m16, st);
    else if (p.T == 2)
      launch_tn<2, 4>(vec, p, rows, m, n, A, lda, B1, B2, n1, ldb, partial, m16, st);
    else
      launch_tn<1, 16>(vec, p, rows, m, n, A, lda, B1, B2, n1, ldb, partial, m16, st);
  }
  STS_HIP(hipGetLastError());
  const int64_t nch = rows <= 0 ? 1 : p.nch;
  launch(STS_K_GRAM_REDUCE, 8.0 * ((double)nch * m16 * 16 + (double)m * n), gemm_tn_reduce,
         dim3((m * n + 3) / 4), dim3(256), 0, st, m, n, nch, m16, (const double*)partial, C1, C2,
         n1, ldc);
}

void gemm_tn(int64_t rows, int m, int n, const double* A, int64_t lda, const double* B,
             int64_t ldb, double* C, int64_t ldc, double* partial, hipStream_t st) {
  gemm_tn2(rows, m, n, 0, A, lda, B, B, ldb, C, C, ldc, partial, st);
}

int64_t gemm_tn_partial_size_wide(int64_t rows, int m) {
  return 2 * gemm_tn_partial_size(rows, m);
}

template <int T, int NW, int NB>
static void launch_tnw(bool vec, const TnPlan& p, int64_t rows, int m, int n, const double* A,
                       int64_t lda, const TnSegs& sg, int64_t ldb, double* partial, int m16,
                       hipStream_t st) {
  const dim3 grid((unsigned)p.groups, (unsigned)p.nch);
  const double bytes = 8.0 * (double)rows * (m + n);
  if (vec)
    launch(STS_K_GRAM, bytes, gemm_tnw_kernel<T, NW, NB, true>, grid, dim3(64 * NW), 0, st, rows,
           m, n, A, lda, sg, ldb, partial, m16, p.rpw);
  else
    launch(STS_K_GRAM, bytes, gemm_tnw_kernel<T, NW, NB, false>, grid, dim3(64 * NW), 0, st, rows,
           m, n, A, lda, sg, ldb, partial, m16, p.rpw);
}

void gemm_tn_segs(int64_t rows, int m, const double* A, int64_t lda, int nseg,
                  const double* const* B, const int* nb, int64_t ldb, double* const* C,
                  const int64_t* ldc, double* partial, hipStream_t st) {
  STS_REQUIRE(nseg >= 1 && nseg <= 3, STS_E_INVALID, "gemm_tn_segs: 1..3 segments");
  TnSegs sg{};
  TnOut out{};
  int n = 0;
  bool vec = aligned16(A) && lda % 2 == 0 && ldb % 2 == 0;
  for (int s = 0; s < 3; ++s) {
    const int w = s < nseg ? nb[s] : 0;
    STS_REQUIRE(w >= 0, STS_E_INVALID, "gemm_tn_segs: negative width");
    n += w;
    sg.B[s] = s < nseg ? B[s] : B[0];
    sg.end[s] = n;
    out.C[s] = s < nseg ? C[s] : C[0];
    out.ldc[s] = s < nseg ? ldc[s] : ldc[0];
    out.end[s] = n;
    if (s < nseg && w > 0) vec = vec && aligned16(B[s]);
  }
  if (m <= 0 || n <= 0) return;
  STS_REQUIRE(n <= 32, STS_E_INVALID, "gemm_tn_segs: more than 32 columns");
  const int NB = n > 16 ? 2 : 1;
  const int width = 16 * NB;
  const int m16 = ((m + 15) / 16) * 16;
  // 32 columns over four tiles: eight waves per work-group, each over half
  // the rows of a four-wave plan (m = 400, 24 columns: 4.5 against 4.3 TB/s)
  const bool wide8 = NB == 2 && (m + 15) / 16 >= 8;
  const TnPlan p = tn_plan(rows, m, wide8 ? 8 : 0);
  if (rows <= 0) {
    fill_kernel<<<1, 256, 0, st>>>(partial, (int64_t)m16 * width, 0.0);
  } else if (NB == 2) {
    if (p.T == 4) launch_tnw<4, 8, 2>(vec, p, rows, m, n, A, lda, sg, ldb, partial, m16, st);
    else if (p.T == 2) launch_tnw<2, 4, 2>(vec, p, rows, m, n, A, lda, sg, ldb, partial, m16, st);
    else launch_tnw<1, 16, 2>(vec, p, rows, m, n, A, lda, sg, ldb, partial, m16, st);
  } else {
    if (p.T == 4) launch_tnw<4, 4, 1>(vec, p, rows, m, n, A, lda, sg, ldb, partial, m16, st);
    else if (p.T == 2) launch_tnw<2, 4, 1>(vec, p, rows, m, n, A, lda, sg, ldb, partial, m16, st);
    else launch_tnw<1, 16, 1>(vec, p, rows, m, n, A, lda, sg, ldb, partial, m16, st);
  }
  STS_HIP(hipGetLastError());
  const int64_t nch = rows <= 0 ? 1 : p.nch;
  launch(STS_K_GRAM_REDUCE, 8.0 * ((double)nch * m16 * width + (double)m * n), gemm_tnw_reduce,
         dim3((m * n + 3) / 4), dim3(256), 0, st, m, n, nch, m16, width, (const double*)partial,
         out);
  STS_HIP(hipGetLastError());
}

void gemm_nn_sub(int64_t rows, int m, int n, const double* A, int64_t lda, const double* C,
                 int64_t ldc, double* W, int64_t ldw, hipStream_t st) {
  if (m <= 0 || n <= 0 || rows <= 0) return;
  STS_REQUIRE(n <= 16, STS_E_INVALID, "gemm_nn_sub: n > 16");
  const double bytes = 8.0 * (double)rows * (m + 2 * n);
  if (rows >= 64 * 1024) {
    // tall blocks: 64 rows per wave, four accumulator chains
    const int64_t blocks = (rows + 255) / 256;
    if (aligned16(A) && lda % 2 == 0)
      launch(STS_K_BASIS_UPDATE, bytes, gemm_nn_sub4_kernel<true>, dim3((unsigned)blocks),
             dim3(256), 0, st, rows, m, n, A, lda, C, ldc, W, ldw);
    else
      launch(STS_K_BASIS_UPDATE, bytes, gemm_nn_sub4_kernel<false>, dim3((unsigned)blocks),
             dim3(256), 0, st, rows, m, n, A, lda, C, ldc, W, ldw);
  } else {
    const int64_t blocks = (rows + 63) / 64;
    launch(STS_K_BASIS_UPDATE, bytes, gemm_nn_sub_kernel, dim3((unsigned)blocks), dim3(256), 0,
           st, rows, m, n, A, lda, C, ldc, W, ldw);
  }
  STS_HIP(hipGetLastError());
}

void gemm_small(bool transA, int m, int n, int kk, double alpha, const double* A, int64_t lda,
                const double* B, int64_t ldb, double beta, double* D, int64_t ldd,
                hipStream_t st) {
  if (m <= 0 || n <= 0) return;
  if (kk <= 0) {
    if (beta != 1.0)
      for (int j = 0; j < n; ++j) scale_kernel<<<(m + 255) / 256, 256, 0, st>>>(D + (int64_t)j * ldd, m, beta);
    STS_HIP(hipGetLastError());
    return;
  }
  const int tiles = ((m + 15) / 16) * ((n + 15) / 16);
  if (transA)
    gemm_small_kernel<true><<<(tiles + 3) / 4, 256, 0, st>>>(m, n, kk, alpha, A, lda, B, ldb,
                                                             beta, D, ldd);
  else
    gemm_small_kernel<false><<<(tiles + 3) / 4, 256, 0, st>>>(m, n, kk, alpha, A, lda, B, ldb,
                                                              beta, D, ldd);
  STS_HIP(hipGetLastError());
}

void gemm_nn(int m, int n, int kk, const double* A, int64_t lda, const double* B, int64_t ldb,
             double* D, int64_t ldd, hipStream_t st) {
  gemm_small(false, m, n, kk, 1.0, A, lda, B, ldb, 0.0, D, ldd, st);
}

int64_t residual_norm2_partial_size(int64_t rows, int n) {
  return ((rows + 63) / 64) * ((n + 255) / 256);
}

void residual_norm2(int64_t rows, int n, const Seg* segs, int nseg, const double* BT,
                    int64_t ldbt, double* out, double* partial, unsigned* counter,
                    hipStream_t st, bool upper) {
  STS_REQUIRE(nseg >= 1 && nseg <= 3, STS_E_INVALID, "residual_norm2: 1..3 segments");
  ResArgs a{};
  a.rows = rows;
  a.n = n;
  a.nseg = nseg;
  int mtot = 0;
  bool vec = true;
  for (int s = 0; s < nseg; ++s) {
    a.A[s] = segs[s].A;
    a.lda[s] = segs[s].lda;
    a.m[s] = segs[s].m;
    mtot += segs[s].m;
    vec = vec && aligned16(segs[s].A) && segs[s].lda % 2 == 0;
  }
  a.BT = BT;
  a.ldbt = ldbt;
  a.upper = upper ? 1 : 0;
  a.partial = partial;
  a.counter = counter;
  a.out = out;
  dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((n + 255) / 256));
  const double bytes = 8.0 * ((double)rows * mtot + (double)n * mtot);
  if (vec)
    launch(STS_K_RESIDUAL, bytes, residual_kernel<true>, grid, dim3(256), 0, st, a);
  else
    launch(STS_K_RESIDUAL, bytes, residual_kernel<false>, grid, dim3(256), 0, st, a);
  STS_HIP(hipGetLastError());
}

void chol_deflate(int b, const double* G, int64_t ldg, const double* norm0, double defl_v,
                  double defl_b, double* Rinv, CholInfo* info, hipStream_t st) {
  STS_REQUIRE(b >= 0 && b <= 16, STS_E_INVALID, "chol_deflate: b > 16");
  chol_deflate_kernel<<<1, 64, 0, st>>>(b, G, ldg, norm0, defl_v, defl_b, Rinv, info);
  STS_HIP(hipGetLastError());
}

void apply_rinv(int64_t rows, int b, const CholInfo* info, const double* Rinv, double* W,
                double* MW, int64_t ldw, double* /*tmp*/, hipStream_t st) {
  if (rows <= 0 || b <= 0) return;
  STS_REQUIRE(b <= 16, STS_E_INVALID, "apply_rinv: b > 16");
  apply_rinv_kernel<<<(unsigned)((rows + 255) / 256), 256, 0, st>>>(rows, b, info, Rinv, W, MW,
                                                                     ldw);
  STS_HIP(hipGetLastError());
}

void copy_cols(int64_t rows, int ncols, const double* src, int64_t lds, double* dst, int64_t ldd,
               hipStream_t st) {
  if (rows <= 0 || ncols <= 0) return;
  const dim3 grid((unsigned)std::min<int64_t>((rows + 255) / 256, 8192),
                  (unsigned)std::min(ncols, 1024));
  copy_cols_kernel<<<grid, 256, 0, st>>>(rows, ncols, src, lds, dst, ldd);
  STS_HIP(hipGetLastError());
}

void scale(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return;
  scale_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, n, v);
  STS_HIP(hipGetLastError());
}

void fill(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return;
  fill_kernel<<<(unsigned)std::min<int64_t>((n + 255) / 256, 65536), 256, 0, st>>>(p, n, v);
  STS_HIP(hipGetLastError());
}

void sumsq(int64_t rows, int ncols, const double* A, int64_t lda, double* out, double* partial,
           unsigned* counter, hipStream_t st) {
  const int64_t total = rows * ncols;
  int blocks = (int)std::min<int64_t>((total + 255) / 256, 1024);
  if (blocks < 1) blocks = 1;
  sumsq_kernel<<<blocks, 256, 0, st>>>(rows, ncols, A, lda, partial, counter, out);
  STS_HIP(hipGetLastError());
}

// FP32 Gram-Schmidt contraction (see the kernels above).
void gemm_tn32(int64_t rows, int m, int n, const float* A, int64_t lda, const double* B,
               int64_t ldb, double* C, int64_t ldc, float* partial, hipStream_t st) {
  if (m <= 0 || n <= 0) return;
  STS_REQUIRE(n <= 16, STS_E_INVALID, "gemm_tn32: n > 16");
  const int m16 = ((m + 15) / 16) * 16;
  const TnPlan p = tn_plan(rows, m);
  if (rows <= 0) {
    fill_kernel<<<1, 256, 0, st>>>(reinterpret_cast<double*>(partial), (int64_t)m16 * 8, 0.0);
  } else {
    const bool vec = aligned16(A) && aligned16(B) && lda % 4 == 0 && ldb % 2 == 0;
    const dim3 grid((unsigned)p.groups, (unsigned)p.nch);
    const double bytes = 4.0 * (double)rows * m + 8.0 * (double)rows * n;
    auto go = [&](auto kern, int nw) {
      launch(STS_K_GRAM, bytes, kern, grid, dim3(64 * nw), 0, st, rows, m, n, A, lda, B, ldb,
             partial, m16, p.rpw);
    };
    if (p.T == 4) {
      if (vec) go(gemm_tn32_kernel<4, 4, true>, 4);
      else go(gemm_tn32_kernel<4, 4, false>, 4);
    } else if (p.T == 2) {
      if (vec) go(gemm_tn32_kernel<2, 4, true>, 4);
      else go(gemm_tn32_kernel<2, 4, false>, 4);
    } else {
      if (vec) go(gemm_tn32_kernel<1, 16, true>, 16);
      else go(gemm_tn32_kernel<1, 16, false>, 16);
    }
  }
  STS_HIP(hipGetLastError());
  const int64_t nch = rows <= 0 ? 1 : p.nch;
  launch(STS_K_GRAM_REDUCE, 4.0 * ((double)nch * m16 * 16) + 8.0 * m * n, gemm_tn32_reduce,
         dim3((m * n + 3) / 4), dim3(256), 0, st, m, n, nch, m16, (const float*)partial, C, ldc);
}

void round_cols(int64_t rows, int ncols, const double* src, int64_t lds, float* dst, int64_t ldd,
                hipStream_t st) {
  if (rows <= 0 || ncols <= 0) return;
  const dim3 grid((unsigned)std::min<int64_t>((rows + 255) / 256, 8192),
                  (unsigned)std::min(ncols, 1024));
  round_cols_kernel<<<grid, 256, 0, st>>>(rows, ncols, src, lds, dst, ldd);
  STS_HIP(hipGetLastError());
}

}  // namespace sts
