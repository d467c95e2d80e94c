// Matrix-free spatial operators and the inner conjugate-gradient solver.
//
// Kx and Mx of the P1 / Q1 discretisations on uniform grids are constant-
// coefficient stencils (Sec. 3, spatial matrices), so "SpMM" here streams the
// vectors and never reads a matrix.
//
// The CG iteration is a single-reduction variant: with w = A r kept implicit,
//   beta_i  = gamma_i / gamma_{i-1},
//   alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1}),
//   gamma_i = (r_i, r_i), delta_i = (A r_i, r_i),
// where the denominator equals (p_i, A p_i) because r_i is orthogonal to
// r_{i-1} and (r_i, A p_{i-1}) = -gamma_i / alpha_{i-1}.  One launch performs
//   p <- r + beta p;  s = A p;  x <- x + alpha p;  r <- r - alpha s;
//   partial sums of gamma' = (r, r) and delta' = (A r, r)
// for a tile: r and p are staged with a two-point halo in LDS, p and then
// r - alpha A p are recomputed on the halo, so neither s nor A r is stored.
// Per grid point and column a launch reads r, p, x and writes them back
// (48 bytes).  r and p are read on a halo that neighbouring work-groups own,
// so each launch writes them to the other buffer of a pair (ping-pong by
// launch parity); x is only touched on the tile itself and is updated in
// place.
//
// Reduction without a serial tail: every work-group of launch k first sums
// the per-tile partials written by launch k-1 (in one fixed order, so all
// groups obtain bitwise identical scalars) while its own tile loads are in
// flight, derives alpha and beta, and work-group 0 records the new state.
// State and partials are double-buffered by launch parity, so no fence,
// atomic or grid barrier is needed: the kernel boundary orders them.
#include <hip/hip_runtime.h>

#include "sts_internal.h"

namespace sts {

namespace {

constexpr int kThreads = 256;

template <int TX, int TY, int TZ>
struct Tile {
  static constexpr int X = TX, Y = TY, Z = TZ;
};
// default tile per dimension
template <int DIM>
struct TileShape;
template <>
struct TileShape<1> : Tile<1024, 1, 1> {};
template <>
struct TileShape<2> : Tile<64, 16, 1> {};
template <>
struct TileShape<3> : Tile<32, 8, 4> {};

struct Coefs {
  double k[27];
  double m[27];
};

struct IterArgs {
  int nx, ny, nz;
  int ntx, nty, ntz;      // tiles per direction
  int ncols;              // columns of the batch (state entries)
  int parity;             // launch index & 1
  int nlaunch;            // columns this launch works on (host's view of the active set)
  int cols[kMaxCols];
  int ops[kMaxCols];
  double* x;
  double* r[2];           // r and p are ping-ponged by launch parity: launch k reads
  double* p[2];           // buffer (k-1) & 1 (tile plus halo) and writes buffer k & 1
  int64_t ld;
  CGScal* scal;           // 2 slots of kMaxCols
  double* partials;       // 2 slots of kMaxCols * max_tiles * 2
  int max_tiles;
  Coefs cf;
};

struct SetupArgs {
  IterArgs it;
  const double* b[kMaxCols];
};

// Work items lin = tile * ncols + column.  Block ids are handed to the 8 XCDs
// round-robin; the remap gives each XCD one contiguous range of work items,
// i.e. a contiguous band of tiles for every column, so halo reads mostly hit
// the XCD's own L2 and the XCDs stay balanced when some columns have stopped.
__device__ __forceinline__ int xcd_remap(int bid, int n) {
  const int q = n >> 3, rem = n & 7;
  const int x = bid & 7, j = bid >> 3;
  return x * q + min(x, rem) + j;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }


template <class T>
__device__ __forceinline__ void tile_origin(const IterArgs& a, int t, int& x0, int& y0, int& z0) {
  const int tx = t % a.ntx;
  const int rest = t / a.ntx;
  x0 = tx * T::X;
  y0 = (rest % a.nty) * T::Y;
  z0 = (rest / a.nty) * T::Z;
}

// Sparsity patterns of the stencils, bit (dz+1)*9 + (dy+1)*3 + (dx+1) per
// neighbour offset; fixed per discretisation so that the stencil loops have
// no run-time branches.
constexpr unsigned kMask1D = (1u << 12) | (1u << 13) | (1u << 14);
constexpr unsigned kMask2DK = (1u << 10) | (1u << 12) | (1u << 13) | (1u << 14) | (1u << 16);
constexpr unsigned kMask2DM = kMask2DK | (1u << 9) | (1u << 17);   // + SW, NE (Courant diagonal)
constexpr unsigned kMask3DK = kMask2DK | (1u << 4) | (1u << 22);
constexpr unsigned kMask3DM = 0x7FFFFFFu;

template <int DIM>
struct Masks;
template <>
struct Masks<1> { static constexpr unsigned K = kMask1D, M = kMask1D; };
template <>
struct Masks<2> { static constexpr unsigned K = kMask2DK, M = kMask2DM; };
template <>
struct Masks<3> { static constexpr unsigned K = kMask3DK, M = kMask3DM; };

// Apply the stencil with pattern MASK at LDS point (ix, iy, iz) of an array
// laid out RX x RY x RZ.
template <unsigned MASK, int RX, int RY>
__device__ __forceinline__ double apply_lds(const double* c, const double* s, int ix, int iy,
                                            int iz) {
  double acc = 0.0;
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int bit = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
        if ((MASK >> bit) & 1u)
          acc += c[bit] * s[((iz + dz) * RY + (iy + dy)) * RX + (ix + dx)];
      }
  return acc;
}

// Sum of (g, d) over a block of NT threads in a fixed order; valid in thread 0.
template <int NT = kThreads>
__device__ __forceinline__ void block_sum2(double& g, double& d, double* red) {
  g = wave_sum(g);
  d = wave_sum(d);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[2 * wv] = g;
    red[2 * wv + 1] = d;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    g = 0.0;
    d = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
      g += red[2 * w];
      d += red[2 * w + 1];
    }
  }
}

// Per-thread share of the previous launch's partials, loaded before the tile
// so that its latency overlaps the tile loads (a wait on a later load would
// also wait on every earlier one).  One tile per thread for the first
// kPreCols launched columns is held in registers; further tiles and columns
// are summed in a loop after the tile loads.  Columns outside the launch list
// have already stopped (the host drops a column only after seeing it stop).
constexpr int kPreCols = 4;

struct Pre {
  double g[kPreCols];
  double d[kPreCols];
  CGScal prev;            // state of launched column threadIdx.x
};

template <int NT>
__device__ __forceinline__ void pre_load(const IterArgs& a, int ntiles, Pre& P) {
  const double* pin = a.partials + (size_t)(a.parity ^ 1) * kMaxCols * a.max_tiles * 2;
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < kPreCols; ++j) {
    P.g[j] = 0.0;
    P.d[j] = 0.0;
    if (j < a.nlaunch && t < ntiles) {
      const double* pp = pin + ((size_t)a.cols[j] * a.max_tiles + t) * 2;
      P.g[j] = pp[0];
      P.d[j] = pp[1];
    }
  }
  if ((int)threadIdx.x < a.nlaunch)
    P.prev = a.scal[(a.parity ^ 1) * kMaxCols + a.cols[threadIdx.x]];
}

// Sum the partials (fixed order), take the CG decisions (thread j for launch
// slot j) and, in work-group 0, record the new state of every column.
template <int NT>
__device__ void step_scalars(const IterArgs& a, int ntiles, bool writer, const Pre& P,
                             double (*red)[NT / 64], double* s_alpha, double* s_beta, int* s_go) {
  const double* pin = a.partials + (size_t)(a.parity ^ 1) * kMaxCols * a.max_tiles * 2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kMaxCols; ++j) {
    if (j >= a.nlaunch) break;
    double g = 0.0, d = 0.0;
    int t0 = threadIdx.x;
    if (j < kPreCols) {
      g = P.g[j];
      d = P.d[j];
      t0 += NT;
    }
    const double* pc = pin + (size_t)a.cols[j] * a.max_tiles * 2;
    for (int t = t0; t < ntiles; t += NT) {
      g += pc[2 * t];
      d += pc[2 * t + 1];
    }
    g = wave_sum(g);
    d = wave_sum(d);
    if (lane == 0) {
      red[2 * j][wv] = g;
      red[2 * j + 1][wv] = d;
    }
  }
  __syncthreads();
  const int j = threadIdx.x;
  if (j < a.nlaunch) {
    CGScal s = P.prev;
    int go = 0;
    double al = 0.0, be = 0.0;
    if (s.active) {
      double g = 0.0, d = 0.0;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) {
        g += red[2 * j][w];
        d += red[2 * j + 1][w];
      }
      if (!finite(g) || !finite(d)) {
        s.active = 0;
        s.flag = 3;
      } else if (s.iters == 0) {
        s.gamma0 = g;
        if (g == 0.0) {
          s.active = 0;
          s.flag = 1;
        } else if (!(d > 0.0)) {
          s.active = 0;
          s.flag = 3;
        } else {
          al = g / d;
          go = 1;
        }
      } else if (g <= s.rtol2 * s.gamma0) {
        s.active = 0;
        s.flag = 1;
      } else if (s.iters >= s.maxit) {
        s.active = 0;
        s.flag = 2;
      } else {
        be = g / s.gamma;
        const double den = d - be * g / s.alpha;
        if (!(den > 0.0)) {
          s.active = 0;
          s.flag = 3;
        } else {
          al = g / den;
          go = 1;
        }
      }
      s.gamma = g;
      if (go) {
        s.alpha = al;
        s.iters += 1;
      }
    }
    s_go[j] = go;
    s_alpha[j] = al;
    s_beta[j] = be;
    if (writer) a.scal[a.parity * kMaxCols + a.cols[j]] = s;
  }
  if (writer && j < a.ncols) {
    bool launched = false;
    for (int q = 0; q < a.nlaunch; ++q) launched |= a.cols[q] == j;
    if (!launched) a.scal[a.parity * kMaxCols + j] = a.scal[(a.parity ^ 1) * kMaxCols + j];
  }
  __syncthreads();
}

// Stages of one CG iteration on one tile, given the loaded r, p (tile plus
// two-point halo) and x (tile) in registers.
template <int DIM, class T, int NT, unsigned MASK, int LR, int LI>
__device__ __forceinline__ void cg_tile_stages(const IterArgs& a, const double* cf, int c, int t,
                                               int x0, int y0, int z0, double alpha, double beta,
                                               const double (&rr)[LR], const double (&pv)[LR],
                                               const double (&xv)[LI], double* rs, double* ps,
                                               double* red) {
  constexpr int H = 2;
  constexpr int RX = T::X + 2 * H;
  constexpr int RY = DIM >= 2 ? T::Y + 2 * H : 1;
  constexpr int RZ = DIM >= 3 ? T::Z + 2 * H : 1;
  constexpr int NR = RX * RY * RZ;
  constexpr int SX = T::X + 2, SY = DIM >= 2 ? T::Y + 2 : 1, SZ = DIM >= 3 ? T::Z + 2 : 1;
  constexpr int NS = SX * SY * SZ;
  constexpr int LS = (NS + NT - 1) / NT;
  constexpr int NI = T::X * T::Y * T::Z;
  constexpr int OY = DIM >= 2 ? 1 : 0, OZ = DIM >= 3 ? 1 : 0;   // S-region offset in R
  constexpr int IY = DIM >= 2 ? 2 : 0, IZ = DIM >= 3 ? 2 : 0;   // interior offset in R
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const size_t sxy = (size_t)nx * ny;
  double* xg = a.x + (size_t)c * a.ld;
  double* rg = a.r[a.parity] + (size_t)c * a.ld;
  double* pg = a.p[a.parity] + (size_t)c * a.ld;

  // stage 1: r and p <- r + beta p on the tile plus a two-point halo
#pragma unroll
  for (int u = 0; u < LR; ++u) {
    const int i = threadIdx.x + u * NT;
    if (i < NR) {
      rs[i] = rr[u];
      ps[i] = rr[u] + beta * pv[u];
    }
  }
  __syncthreads();

  // stage 2: on the tile plus a one-point halo, r <- r - alpha A p (zero outside);
  // all reads of this stage come from ps, so its iterations are independent
  double sv[LS];
#pragma unroll
  for (int u = 0; u < LS; ++u) {
    const int i = threadIdx.x + u * NT;
    sv[u] = 0.0;
    if (i < NS) {
      const int sx = i % SX, sy = (i / SX) % SY, sz = i / (SX * SY);
      sv[u] = apply_lds<MASK, RX, RY>(cf, ps, sx + 1, sy + OY, sz + OZ);
    }
  }
#pragma unroll
  for (int u = 0; u < LS; ++u) {
    const int i = threadIdx.x + u * NT;
    if (i < NS) {
      const int sx = i % SX, sy = (i / SX) % SY, sz = i / (SX * SY);
      const int gx = x0 - 1 + sx;
      const int gy = DIM >= 2 ? y0 - 1 + sy : 0;
      const int gz = DIM >= 3 ? z0 - 1 + sz : 0;
      const int q = ((sz + OZ) * RY + (sy + OY)) * RX + (sx + 1);
      const bool in = gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
      rs[q] = in ? rs[q] - alpha * sv[u] : 0.0;
    }
  }
  __syncthreads();

  // stage 3: interior -- gamma', delta' partials; write x, r, p
  double gsum = 0.0, dsum = 0.0;
#pragma unroll
  for (int u = 0; u < LI; ++u) {
    const int i = threadIdx.x + u * NT;
    if (i < NI) {
      const int ux = i % T::X, uy = (i / T::X) % T::Y, uz = i / (T::X * T::Y);
      const int gx = x0 + ux, gy = y0 + uy, gz = z0 + uz;
      if (gx < nx && gy < ny && gz < nz) {
        const int ix = ux + 2, iy = uy + IY, iz = uz + IZ;
        const int q = (iz * RY + iy) * RX + ix;
        const double w = apply_lds<MASK, RX, RY>(cf, rs, ix, iy, iz);
        const double rn = rs[q];
        const double pn = ps[q];
        gsum += rn * rn;
        dsum += w * rn;
        const size_t gi = (size_t)gz * sxy + (size_t)gy * nx + gx;
        xg[gi] = xv[u] + alpha * pn;
        rg[gi] = rn;
        pg[gi] = pn;
      }
    }
  }
  __syncthreads();   // red[] reuse
  block_sum2<NT>(gsum, dsum, red);
  if (threadIdx.x == 0) {
    double* po = a.partials + ((size_t)a.parity * kMaxCols * a.max_tiles + (size_t)c * a.max_tiles +
                               t) * 2;
    po[0] = gsum;
    po[1] = dsum;
  }
}

template <int DIM, class T = TileShape<DIM>, int NT = kThreads>
__global__ __launch_bounds__(NT) void cg_iter_kernel(IterArgs a) {
  constexpr int H = 2;
  constexpr int RX = T::X + 2 * H;
  constexpr int RY = DIM >= 2 ? T::Y + 2 * H : 1;
  constexpr int RZ = DIM >= 3 ? T::Z + 2 * H : 1;
  constexpr int NR = RX * RY * RZ;
  constexpr int LR = (NR + NT - 1) / NT;
  constexpr int NI = T::X * T::Y * T::Z;
  constexpr int LI = (NI + NT - 1) / NT;

  __shared__ double rs[NR];
  __shared__ double ps[NR];
  __shared__ double red[2 * kMaxCols][NT / 64];
  __shared__ double s_alpha[kMaxCols], s_beta[kMaxCols];
  __shared__ int s_go[kMaxCols];

  const int ntiles = a.ntx * a.nty * a.ntz;
  const int lin = xcd_remap(blockIdx.x, a.nlaunch * ntiles);
  const int t = lin / a.nlaunch, jb = lin % a.nlaunch, c = a.cols[jb];
  const bool writer = blockIdx.x == 0;

  Pre pre;
  pre_load<NT>(a, ntiles, pre);

  int x0, y0, z0;
  tile_origin<T>(a, t, x0, y0, z0);
  const double* xg = a.x + (size_t)c * a.ld;
  const double* rg = a.r[a.parity ^ 1] + (size_t)c * a.ld;
  const double* pg = a.p[a.parity ^ 1] + (size_t)c * a.ld;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const size_t sxy = (size_t)nx * ny;

  // issue every global load of the tile before waiting on the scalars
  double rr[LR], pv[LR], xv[LI];
  {
#pragma unroll
    for (int u = 0; u < LR; ++u) {
      const int i = threadIdx.x + u * NT;
      rr[u] = 0.0;
      pv[u] = 0.0;
      if (i < NR) {
        const int lx = i % RX, ly = (i / RX) % RY, lz = i / (RX * RY);
        const int gx = x0 - H + lx;
        const int gy = DIM >= 2 ? y0 - H + ly : 0;
        const int gz = DIM >= 3 ? z0 - H + lz : 0;
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz) {
          const size_t gi = (size_t)gz * sxy + (size_t)gy * nx + gx;
          rr[u] = rg[gi];
          pv[u] = pg[gi];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < LI; ++u) {
      const int i = threadIdx.x + u * NT;
      xv[u] = 0.0;
      if (i < NI) {
        const int gx = x0 + i % T::X, gy = y0 + (i / T::X) % T::Y, gz = z0 + i / (T::X * T::Y);
        if (gx < nx && gy < ny && gz < nz) xv[u] = xg[(size_t)gz * sxy + (size_t)gy * nx + gx];
      }
    }
  }

  step_scalars<NT>(a, ntiles, writer, pre, red, s_alpha, s_beta, s_go);
  if (!s_go[jb]) return;
  const double alpha = s_alpha[jb];
  const double beta = s_beta[jb];
  if (a.ops[c])
    cg_tile_stages<DIM, T, NT, Masks<DIM>::M>(a, a.cf.m, c, t, x0, y0, z0, alpha, beta, rr, pv, xv,
                                               rs, ps, &red[0][0]);
  else
    cg_tile_stages<DIM, T, NT, Masks<DIM>::K>(a, a.cf.k, c, t, x0, y0, z0, alpha, beta, rr, pv, xv,
                                               rs, ps, &red[0][0]);
}

template <int DIM, class T = TileShape<DIM>>
__global__ __launch_bounds__(kThreads) void cg_setup_kernel(SetupArgs sa) {
  const IterArgs& a = sa.it;
  constexpr int H = 1;
  constexpr int RX = T::X + 2 * H;
  constexpr int RY = DIM >= 2 ? T::Y + 2 * H : 1;
  constexpr int RZ = DIM >= 3 ? T::Z + 2 * H : 1;
  constexpr int NR = RX * RY * RZ;
  constexpr int NI = T::X * T::Y * T::Z;
  constexpr int IY = DIM >= 2 ? 1 : 0, IZ = DIM >= 3 ? 1 : 0;

  __shared__ double bs[NR];
  __shared__ double red[8];

  const int ntiles = a.ntx * a.nty * a.ntz;
  const int lin = xcd_remap(blockIdx.x, a.ncols * ntiles);
  const int t = lin / a.ncols, c = lin % a.ncols;
  if (!a.scal[c].active) return;     // the host wrote the initial state to slot 0
  int x0, y0, z0;
  tile_origin<T>(a, t, x0, y0, z0);
  const double* cf = a.ops[c] ? a.cf.m : a.cf.k;
  const double* bg = sa.b[c];
  double* xg = a.x + (size_t)c * a.ld;
  double* rg = a.r[0] + (size_t)c * a.ld;     // the set-up is launch 0
  double* pg = a.p[0] + (size_t)c * a.ld;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const size_t sxy = (size_t)nx * ny;

  for (int i = threadIdx.x; i < NR; i += kThreads) {
    const int lx = i % RX, ly = (i / RX) % RY, lz = i / (RX * RY);
    const int gx = x0 - H + lx;
    const int gy = DIM >= 2 ? y0 - H + ly : 0;
    const int gz = DIM >= 3 ? z0 - H + lz : 0;
    double v = 0.0;
    if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz)
      v = bg[(size_t)gz * sxy + (size_t)gy * nx + gx];
    bs[i] = v;
  }
  __syncthreads();
  double gsum = 0.0, dsum = 0.0;
  for (int i = threadIdx.x; i < NI; i += kThreads) {
    const int ux = i % T::X, uy = (i / T::X) % T::Y, uz = i / (T::X * T::Y);
    const int gx = x0 + ux, gy = y0 + uy, gz = z0 + uz;
    if (gx < nx && gy < ny && gz < nz) {
      const int ix = ux + 1, iy = uy + IY, iz = uz + IZ;
      const double bv = bs[(iz * RY + iy) * RX + ix];
      const double w = a.ops[c] ? apply_lds<Masks<DIM>::M, RX, RY>(cf, bs, ix, iy, iz)
                                : apply_lds<Masks<DIM>::K, RX, RY>(cf, bs, ix, iy, iz);
      gsum += bv * bv;
      dsum += w * bv;
      const size_t gi = (size_t)gz * sxy + (size_t)gy * nx + gx;
      xg[gi] = 0.0;
      rg[gi] = bv;
      pg[gi] = 0.0;
    }
  }
  block_sum2(gsum, dsum, red);
  if (threadIdx.x == 0) {
    double* po = a.partials + ((size_t)c * a.max_tiles + t) * 2;   // slot 0
    po[0] = gsum;
    po[1] = dsum;
  }
}

__global__ void cg_init_state_kernel(CGScal* scal, int ncols, double rtol2, int maxit) {
  const int c = threadIdx.x;
  if (c >= kMaxCols) return;
  CGScal s{};
  s.rtol2 = rtol2;
  s.maxit = maxit;
  s.active = c < ncols ? 1 : 0;
  scal[c] = s;                  // slot 0
  scal[kMaxCols + c] = s;       // slot 1 (never read before it is written)
}

struct ApplyArgs {
  int nx, ny, nz, ntx, nty, ntz, ncols;
  int ops[16];
  const double* X;
  int64_t ldx;
  double* Y;
  int64_t ldy;
  double* Y2;     // non-null: Y = Kx X and Y2 = Mx X from one read of X (ops ignored)
  int64_t ldy2;
  Coefs cf;
};

template <int DIM>
__global__ __launch_bounds__(kThreads) void apply_kernel(ApplyArgs a) {
  using T = TileShape<DIM>;
  constexpr int H = 1;
  constexpr int RX = T::X + 2 * H;
  constexpr int RY = DIM >= 2 ? T::Y + 2 * H : 1;
  constexpr int RZ = DIM >= 3 ? T::Z + 2 * H : 1;
  constexpr int NR = RX * RY * RZ;
  constexpr int NI = T::X * T::Y * T::Z;
  constexpr int IY = DIM >= 2 ? 1 : 0, IZ = DIM >= 3 ? 1 : 0;
  __shared__ double xs[NR];

  const int ntiles = a.ntx * a.nty * a.ntz;
  const int lin = xcd_remap(blockIdx.x, ntiles * a.ncols);
  const int t = lin / a.ncols, c = lin % a.ncols;
  const int tx = t % a.ntx, ty = (t / a.ntx) % a.nty, tz = t / (a.ntx * a.nty);
  const int x0 = tx * T::X, y0 = ty * T::Y, z0 = tz * T::Z;
  const double* cf = a.ops[c] ? a.cf.m : a.cf.k;
  const double* xg = a.X + (size_t)c * a.ldx;
  double* yg = a.Y + (size_t)c * a.ldy;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const size_t sxy = (size_t)nx * ny;
  {
    // all of a thread's halo loads in flight together: branch-free (outside
    // the domain the load reads the column's first node and the value is
    // dropped), fully unrolled, stored to LDS after the last one is issued
    constexpr int NL = (NR + kThreads - 1) / kThreads;
    double v[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int i = min((int)threadIdx.x + k * kThreads, NR - 1);
      const int lx = i % RX, ly = (i / RX) % RY, lz = i / (RX * RY);
      const int gx = x0 - H + lx;
      const int gy = DIM >= 2 ? y0 - H + ly : 0;
      const int gz = DIM >= 3 ? z0 - H + lz : 0;
      const bool in = gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
      const double x = xg[in ? (size_t)gz * sxy + (size_t)gy * nx + gx : 0];
      v[k] = in ? x : 0.0;
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int i = threadIdx.x + k * kThreads;
      if (i < NR) xs[i] = v[k];
    }
  }
  __syncthreads();
  if (a.Y2) {
    // both images of the column from the one LDS tile
    double* y2 = a.Y2 + (size_t)c * a.ldy2;
    for (int i = threadIdx.x; i < NI; i += kThreads) {
      const int ux = i % T::X, uy = (i / T::X) % T::Y, uz = i / (T::X * T::Y);
      const int gx = x0 + ux, gy = y0 + uy, gz = z0 + uz;
      if (gx < nx && gy < ny && gz < nz) {
        const size_t g = (size_t)gz * sxy + (size_t)gy * nx + gx;
        yg[g] = apply_lds<Masks<DIM>::K, RX, RY>(a.cf.k, xs, ux + 1, uy + IY, uz + IZ);
        y2[g] = apply_lds<Masks<DIM>::M, RX, RY>(a.cf.m, xs, ux + 1, uy + IY, uz + IZ);
      }
    }
    return;
  }
  for (int i = threadIdx.x; i < NI; i += kThreads) {
    const int ux = i % T::X, uy = (i / T::X) % T::Y, uz = i / (T::X * T::Y);
    const int gx = x0 + ux, gy = y0 + uy, gz = z0 + uz;
    if (gx < nx && gy < ny && gz < nz)
      yg[(size_t)gz * sxy + (size_t)gy * nx + gx] =
          a.ops[c] ? apply_lds<Masks<DIM>::M, RX, RY>(cf, xs, ux + 1, uy + IY, uz + IZ)
                   : apply_lds<Masks<DIM>::K, RX, RY>(cf, xs, ux + 1, uy + IY, uz + IZ);
  }
}

template <int DIM>
void tiles_of(const Grid& g, int& ntx, int& nty, int& ntz) {
  using T = TileShape<DIM>;
  ntx = (g.nx + T::X - 1) / T::X;
  nty = (g.ny + T::Y - 1) / T::Y;
  ntz = (g.nz + T::Z - 1) / T::Z;
}

void tiles_any(const Grid& g, int& ntx, int& nty, int& ntz) {
  if (g.dim == 1) tiles_of<1>(g, ntx, nty, ntz);
  else if (g.dim == 2) tiles_of<2>(g, ntx, nty, ntz);
  else tiles_of<3>(g, ntx, nty, ntz);
}

IterArgs make_iter_args(const Grid& g, const Stencil& K, const Stencil& M, const int* ops,
                        int ncols, const CGWork& w, int parity) {
  IterArgs a{};
  a.nlaunch = ncols;
  for (int c = 0; c < kMaxCols; ++c) a.cols[c] = c < ncols ? c : 0;
  a.nx = g.nx;
  a.ny = g.ny;
  a.nz = g.nz;
  tiles_any(g, a.ntx, a.nty, a.ntz);
  a.ncols = ncols;
  a.parity = parity;
  for (int c = 0; c < ncols; ++c) a.ops[c] = ops[c];
  a.x = w.x;
  a.r[0] = w.r[0];
  a.r[1] = w.r[1];
  a.p[0] = w.p[0];
  a.p[1] = w.p[1];
  a.ld = w.ld;
  a.scal = w.scal;
  a.partials = w.partials;
  a.max_tiles = w.max_tiles;
  for (int i = 0; i < 27; ++i) {
    a.cf.k[i] = K.c[i];
    a.cf.m[i] = M.c[i];
  }
  return a;
}

// The kernels only visit the offsets of their dimension's patterns.
void check_patterns(const Grid& g, const Stencil& K, const Stencil& M) {
  const unsigned mk = g.dim == 1 ? kMask1D : g.dim == 2 ? kMask2DK : kMask3DK;
  const unsigned mm = g.dim == 1 ? kMask1D : g.dim == 2 ? kMask2DM : kMask3DM;
  for (int b = 0; b < 27; ++b) {
    STS_REQUIRE(((mk >> b) & 1u) || K.c[b] == 0.0, STS_E_INVALID, "stiffness stencil pattern");
    STS_REQUIRE(((mm >> b) & 1u) || M.c[b] == 0.0, STS_E_INVALID, "mass stencil pattern");
  }
}

}  // namespace

int cg_tiles(const Grid& g) {
  int a, b, c;
  tiles_any(g, a, b, c);
  return a * b * c;
}

void cg_init_state(const CGWork& w, int ncols, double rtol, int maxit, hipStream_t st) {
  cg_init_state_kernel<<<1, 64, 0, st>>>(w.scal, ncols, rtol * rtol, maxit);
  STS_HIP(hipGetLastError());
}

void cg_setup(const Grid& g, const Stencil& K, const Stencil& M, const int* ops, int ncols,
              const CGWork& w, hipStream_t st) {
  STS_REQUIRE(ncols >= 1 && ncols <= kMaxCols, STS_E_INVALID, "cg_setup: 1..8 columns");
  STS_REQUIRE(cg_tiles(g) <= w.max_tiles, STS_E_INVALID, "cg_setup: partial buffer too small");
  check_patterns(g, K, M);
  SetupArgs sa;
  sa.it = make_iter_args(g, K, M, ops, ncols, w, 0);
  for (int c = 0; c < kMaxCols; ++c) sa.b[c] = c < ncols ? w.b[c] : nullptr;
  const int blocks = cg_tiles(g) * ncols;
  if (g.dim == 1) cg_setup_kernel<1><<<blocks, kThreads, 0, st>>>(sa);
  else if (g.dim == 2) cg_setup_kernel<2><<<blocks, kThreads, 0, st>>>(sa);
  else cg_setup_kernel<3><<<blocks, kThreads, 0, st>>>(sa);
  STS_HIP(hipGetLastError());
}

void cg_iterate(const Grid& g, const Stencil& K, const Stencil& M, const int* ops, int ncols,
                const CGWork& w, int parity, const int* cols, int nlaunch, hipStream_t st) {
  STS_REQUIRE(nlaunch >= 1 && nlaunch <= ncols, STS_E_INVALID, "cg_iterate: bad launch list");
  IterArgs a = make_iter_args(g, K, M, ops, ncols, w, parity & 1);
  a.nlaunch = nlaunch;
  for (int j = 0; j < nlaunch; ++j) {
    STS_REQUIRE(cols[j] >= 0 && cols[j] < ncols, STS_E_INVALID, "cg_iterate: bad column");
    a.cols[j] = cols[j];
  }
  const int blocks = cg_tiles(g) * nlaunch;
  const double by = 48.0 * (double)g.nh * nlaunch;
  if (g.dim == 1) launch(STS_K_CG_ITER, by, cg_iter_kernel<1>, dim3(blocks), dim3(kThreads), 0, st, a);
  else if (g.dim == 2)
    launch(STS_K_CG_ITER, by, cg_iter_kernel<2>, dim3(blocks), dim3(kThreads), 0, st, a);
  else launch(STS_K_CG_ITER, by, cg_iter_kernel<3>, dim3(blocks), dim3(kThreads), 0, st, a);
  STS_HIP(hipGetLastError());
}

void stencil_apply(const Grid& g, const Stencil& K, const Stencil& M, const int* ops, int ncols,
                   const double* X, int64_t ldx, double* Y, int64_t ldy, hipStream_t st) {
  if (ncols <= 0) return;
  STS_REQUIRE(ncols <= 16, STS_E_INVALID, "stencil_apply: at most 16 columns");
  check_patterns(g, K, M);
  ApplyArgs a{};
  a.nx = g.nx;
  a.ny = g.ny;
  a.nz = g.nz;
  tiles_any(g, a.ntx, a.nty, a.ntz);
  a.ncols = ncols;
  for (int c = 0; c < ncols; ++c) a.ops[c] = ops[c];
  a.X = X;
  a.ldx = ldx;
  a.Y = Y;
  a.ldy = ldy;
  for (int i = 0; i < 27; ++i) {
    a.cf.k[i] = K.c[i];
    a.cf.m[i] = M.c[i];
  }
  const int blocks = a.ntx * a.nty * a.ntz * ncols;
  const double by = 16.0 * (double)g.nh * ncols;
  if (g.dim == 1) launch(STS_K_STENCIL, by, apply_kernel<1>, dim3(blocks), dim3(kThreads), 0, st, a);
  else if (g.dim == 2)
    launch(STS_K_STENCIL, by, apply_kernel<2>, dim3(blocks), dim3(kThreads), 0, st, a);
  else launch(STS_K_STENCIL, by, apply_kernel<3>, dim3(blocks), dim3(kThreads), 0, st, a);
  STS_HIP(hipGetLastError());
}

void stencil_apply_km(const Grid& g, const Stencil& K, const Stencil& M, int ncols,
                      const double* X, int64_t ldx, double* KX, int64_t ldk, double* MX,
                      int64_t ldm, hipStream_t st) {
  if (ncols <= 0) return;
  STS_REQUIRE(ncols <= 16, STS_E_INVALID, "stencil_apply_km: at most 16 columns");
  check_patterns(g, K, M);
  ApplyArgs a{};
  a.nx = g.nx;
  a.ny = g.ny;
  a.nz = g.nz;
  tiles_any(g, a.ntx, a.nty, a.ntz);
  a.ncols = ncols;
  a.X = X;
  a.ldx = ldx;
  a.Y = KX;
  a.ldy = ldk;
  a.Y2 = MX;
  a.ldy2 = ldm;
  for (int i = 0; i < 27; ++i) {
    a.cf.k[i] = K.c[i];
    a.cf.m[i] = M.c[i];
  }
  const int blocks = a.ntx * a.nty * a.ntz * ncols;
  const double by = 24.0 * (double)g.nh * ncols;
  if (g.dim == 1) launch(STS_K_STENCIL, by, apply_kernel<1>, dim3(blocks), dim3(kThreads), 0, st, a);
  else if (g.dim == 2)
    launch(STS_K_STENCIL, by, apply_kernel<2>, dim3(blocks), dim3(kThreads), 0, st, a);
  else launch(STS_K_STENCIL, by, apply_kernel<3>, dim3(blocks), dim3(kThreads), 0, st, a);
  STS_HIP(hipGetLastError());
}

}  // namespace sts
