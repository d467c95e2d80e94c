// Multigrid-preconditioned conjugate gradients for the 2-D P1 stiffness.
//
// The inner solves with Kx (the negative powers of the extended Krylov space,
// Sec. 4) dominate the solver, and unpreconditioned CG needs O(1/h)
// iterations for them.  On the uniform Courant triangulation the P1 spaces of
// the meshes h, 2h, 4h, ... are nested: the prolongation P is P1
// interpolation (coarse values at coincident nodes, the mean of the two end
// points at midpoints of horizontal, vertical and SW-NE edges) and the
// Galerkin coarse operator P^T Kx P is again mu (4; -1, -1, -1, -1) on the
// coarse mesh.
//
// The preconditioner is one V-cycle started from zero:
//  - smoothing: kNu steps of Chebyshev iteration on D^{-1} Kx (D = 4 mu)
//    for the interval [1/2, 2] of its spectrum, before and after each coarse
//    correction (the same polynomial both times, so the two are adjoint);
//  - restriction P^T of the residual, prolongation P of the correction;
//  - the fine levels run as tiled launches; the coarsest level is solved
//    exactly by the fast sine transform: with T = tridiag(-1, 2, -1) =
//    S diag(l) S (S the orthonormal, symmetric DST-I matrix),
//    Kx U = mu (T U + U T) for the nodal array U, so
//    U = S [(S B S) / (mu (l_y + l_x))] S -- four GEMMs on the matrix cores,
//    in one work-group per column up to kMGCoarseMax nodes per direction,
//    over many work-groups up to kMGExactMax.  Grids above kMGCoarseMax keep
//    at least one smoothed level, grids above kMGExactMax halve until the
//    coarsest level fits.
// The V-cycle is a fixed symmetric positive definite operator, so the outer
// iteration is ordinary preconditioned CG.
//
// Launches per PCG iteration: per tiled level a "down" (smoothing from
// zero, residual, restriction -- recomputed on LDS halos; the restricted
// right-hand side and the pre-smoothed iterate on the tile's own nodes are
// stored) and an "up" (pre-smoothed iterate loaded with the halo its kNu
// smoothing steps need, interpolated correction, smoothing), one
// coarse launch, and two PCG launches: A {beta from (r, z); p = z + beta p;
// q = K p; (p, q)} and B {alpha = rho / (p, q); x += alpha p; r -= alpha q;
// (r, r)}.  Global sums are per-tile partials that the consuming work-groups
// add in the same fixed order, so they all take the same decision without
// atomics or a grid barrier.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fst.h"
#include "mg_common.h"
#include "sts_internal.h"

namespace sts {

namespace {

using namespace mgc;

constexpr int kT = 256;          // threads per work-group of the PCG kernels
// Threads per work-group of the level (smoothing) kernels: their LDS regions
// allow two (up) or three (down) work-groups per CU, and 512 threads double
// the waves that hide each work-group's serial smoothing steps.
constexpr int kLT = 512;
constexpr int CX = 32, CY = 8;   // coarse nodes per level-kernel tile (fine footprint 64 x 16)
constexpr int TX = 64, TY = 16;  // fine nodes per PCG-kernel tile
constexpr int kNu = kMGNu;       // smoothing steps
constexpr int kCT = 1024;        // threads of the coarse kernel

// The level operator Kx + s Mx on the Courant triangulation: mu (4; -1 x 4)
// plus s w (6; 1 at W, E, S, N, SW, NE), w = h^2 / 12 of the level.  Both
// matrices are Galerkin products of nested P1 spaces, so every coarse level
// carries the same form with its own w (four times the finer one).
struct Op {
  double mu;           // stiffness coefficient (every level)
  double c0, cx, cd;   // shifted: centre, axis neighbours, SW-NE neighbours
};

// Op applied at LDS point q of an array of row width W; SH = false is the
// unshifted stiffness mu (4 u - u_W - u_E - u_S - u_N).
template <bool SH>
__device__ __forceinline__ double aop(const double* s, int q, int W, const Op& o) {
  if (!SH) return o.mu * (4.0 * s[q] - (s[q - 1] + s[q + 1]) - (s[q - W] + s[q + W]));
  return o.c0 * s[q] + o.cx * ((s[q - 1] + s[q + 1]) + (s[q - W] + s[q + W])) +
         o.cd * (s[q - W - 1] + s[q + W + 1]);
}

template <bool SH>
__device__ __forceinline__ double op_diag(const Op& o) {
  return SH ? o.c0 : 4.0 * o.mu;
}

// P1 interpolation at fine node (gx, gy) from a coarse array with origin
// (cox, coy) and row width CW.  Fine index 2I+1 coincides with coarse I; an
// even fine index 2I+2 lies between coarse I and I+1.
__device__ __forceinline__ double interp(const double* ec, int CW, int cox, int coy, int gx,
                                         int gy) {
  const bool odx = gx & 1, ody = gy & 1;
  const int I = odx ? (gx - 1) >> 1 : (gx >> 1) - 1;
  const int J = ody ? (gy - 1) >> 1 : (gy >> 1) - 1;
  const double* c = ec + (J - coy) * CW + (I - cox);
  if (odx && ody) return c[0];
  if (ody) return 0.5 * (c[0] + c[1]);        // horizontal edge
  if (odx) return 0.5 * (c[0] + c[CW]);       // vertical edge
  return 0.5 * (c[0] + c[CW + 1]);            // SW-NE diagonal edge
}

// An LDS region of W x H fine nodes with global origin (ox, oy) on an n x n
// grid; `shrink` excludes a band at the region's edge (where neighbours are
// missing), nodes outside the domain are excluded (they stay zero).
template <int W, int H>
struct Region {
  int ox, oy, n;
  __device__ __forceinline__ bool inside(int i, int shrink) const {
    const int lx = i % W, ly = i / W;
    const int gx = ox + lx, gy = oy + ly;
    return lx >= shrink && lx < W - shrink && ly >= shrink && ly < H - shrink && gx >= 0 &&
           gx < n && gy >= 0 && gy < n;
  }
};

// One smoothing step with ping-pong buffers: d = a d + c (b - K u) / D and
// u' = u + d on the nodes at least `shrink` inside the region; one barrier.
template <bool SH, int W, int H>
__device__ __forceinline__ void cheb_step(const Region<W, H>& R, int shrink, double ak, double ck,
                                          double inv_d, const double* bs, const double* u,
                                          double* un, double* ds, const Op& op) {
  for (int i = threadIdx.x; i < W * H; i += kLT) {
    if (R.inside(i, shrink)) {
      const double d = ak * ds[i] + ck * inv_d * (bs[i] - aop<SH>(u, i, W, op));
      ds[i] = d;
      un[i] = u[i] + d;
    }
  }
  __syncthreads();
}

// kNu steps from u = 0; step k on shrink k.  Returns the buffer index of u,
// which is valid on shrink kNu - 1.
template <bool SH, int W, int H>
__device__ __forceinline__ int presmooth(const Region<W, H>& R, const Smooth& sm, double inv_d,
                                         const double* bs, double (*us)[W * H], double* ds,
                                         const Op& op) {
  for (int i = threadIdx.x; i < W * H; i += kLT) {
    const double v = R.inside(i, 0) ? sm.c[0] * inv_d * bs[i] : 0.0;
    ds[i] = v;
    us[0][i] = v;
    us[1][i] = v;   // keeps zeros outside the domain in both buffers
  }
  __syncthreads();
  int cur = 0;
  for (int k = 1; k < kNu; ++k) {
    cheb_step<SH, W, H>(R, k, sm.a[k], sm.c[k], inv_d, bs, us[cur], us[cur ^ 1], ds, op);
    cur ^= 1;
  }
  return cur;
}

struct LevelArgs {
  int nf, nc;          // fine / coarse nodes per direction (nf = 2 nc + 1)
  int64_t ldf, ldc;    // column strides
  const double* bf;    // fine right-hand side
  double* bc;          // down: restricted residual
  const double* ec;    // up: coarse correction
  double* ef;          // up: result on the fine level
  double* xp;          // pre-smoothed fine iterate: written by down, read by up
  int ntx, nty;        // coarse tiles
  int nlaunch;
  int cols[kMaxCols];
  const CGScal* st;    // per-column activity, may be null (all active)
  Op op;               // operator of the fine level
  Smooth sm;
  double* part;        // up: per-tile (b, e), may be null
  int max_tiles;
};

// ---------------------------------------------------------------------------
// down: u = smoothing from zero; res = b - K u; b_c = P^T res at the tile's
// coarse nodes.  Fine region [2 cx0 - kNu, 2 cx0 + 2 CX + kNu] per direction.
// ---------------------------------------------------------------------------
template <bool SH>
__global__ __launch_bounds__(kLT) void mg_down_kernel(LevelArgs a) {
  constexpr int W = 2 * CX + 1 + 2 * kNu, H = 2 * CY + 1 + 2 * kNu;
  __shared__ double bs[W * H];
  __shared__ double us[2][W * H];
  __shared__ double ds[W * H];
  const int ntiles = a.ntx * a.nty;
  const int lin = xcd_remap(blockIdx.x, a.nlaunch * ntiles);
  const int t = lin / a.nlaunch, col = a.cols[lin % a.nlaunch];
  if (a.st && !a.st[col].active) return;
  const int cx0 = (t % a.ntx) * CX, cy0 = (t / a.ntx) * CY;
  const int nf = a.nf, nc = a.nc;
  const Region<W, H> R{2 * cx0 - kNu, 2 * cy0 - kNu, nf};
  const Op op = a.op;
  const double inv_d = 1.0 / op_diag<SH>(op);
  const double* bf = a.bf + (size_t)col * a.ldf;
  {
    StagedN<W * H, double, kLT> hb;
    hb.load([&](int i) {
      const int gx = R.ox + i % W, gy = R.oy + i / W;
      return ld_or_zero(bf, gx >= 0 && gx < nf && gy >= 0 && gy < nf, (size_t)gy * nf + gx);
    });
    hb.store(bs);
  }
  __syncthreads();
  const int cur = presmooth<SH, W, H>(R, a.sm, inv_d, bs, us, ds, op);
  // the pre-smoothed iterate on the tile's own fine nodes, for the up launch
  {
    const int x1 = (cx0 + CX >= nc) ? nf : 2 * (cx0 + CX);
    const int y1 = (cy0 + CY >= nc) ? nf : 2 * (cy0 + CY);
    const int ow = x1 - 2 * cx0, oh = y1 - 2 * cy0;
    double* xpg = a.xp + (size_t)col * a.ldf;
    for (int i = threadIdx.x; i < ow * oh; i += kLT) {
      const int gx = 2 * cx0 + i % ow, gy = 2 * cy0 + i / ow;
      xpg[(size_t)gy * nf + gx] = us[cur][(gy - R.oy) * W + (gx - R.ox)];
    }
  }
  // residual on shrink kNu into ds
  for (int i = threadIdx.x; i < W * H; i += kLT) {
    const int lx = i % W, ly = i / W;
    if (lx >= kNu && lx < W - kNu && ly >= kNu && ly < H - kNu)
      ds[i] = bs[i] - aop<SH>(us[cur], i, W, op);
  }
  __syncthreads();
  double* bc = a.bc + (size_t)col * a.ldc;
  for (int i = threadIdx.x; i < CX * CY; i += kLT) {
    const int I = cx0 + i % CX, J = cy0 + i / CX;
    if (I < nc && J < nc) {
      const int q = (2 * (J - cy0) + 1 + kNu) * W + (2 * (I - cx0) + 1 + kNu);
      bc[(size_t)J * nc + I] =
          ds[q] + 0.5 * ((ds[q - 1] + ds[q + 1]) + (ds[q - W] + ds[q + W]) +
                         (ds[q - W - 1] + ds[q + W + 1]));
    }
  }
}

// ---------------------------------------------------------------------------
// up: u = pre-smoothed u (recomputed) + P e_c; smoothing; e on the tile's
// fine nodes [2 cx0, x1) x [2 cy0, y1) (the last tile in a direction runs to
// nf).  Fine region [2 cx0 - (2 kNu - 1), ...), coarse [cx0 - kNu, ...).
// ---------------------------------------------------------------------------
template <bool SH>
__global__ __launch_bounds__(kLT) void mg_up_kernel(LevelArgs a) {
  constexpr int HL = kNu;   // halo of the kNu post-smoothing steps
  constexpr int W = 2 * CX + 1 + 2 * HL, H = 2 * CY + 1 + 2 * HL;
  constexpr int EW = CX + 2 * kNu, EH = CY + 2 * kNu;
  __shared__ double bs[W * H];
  __shared__ double us[2][W * H];
  __shared__ double ds[W * H];
  __shared__ double es[EW * EH];
  __shared__ double red[kLT / 64];
  const int ntiles = a.ntx * a.nty;
  const int lin = xcd_remap(blockIdx.x, a.nlaunch * ntiles);
  const int t = lin / a.nlaunch, col = a.cols[lin % a.nlaunch];
  if (a.st && !a.st[col].active) return;
  const int cx0 = (t % a.ntx) * CX, cy0 = (t / a.ntx) * CY;
  const int nf = a.nf, nc = a.nc;
  const Region<W, H> R{2 * cx0 - HL, 2 * cy0 - HL, nf};
  const int cox = cx0 - kNu, coy = cy0 - kNu;
  const Op op = a.op;
  const double inv_d = 1.0 / op_diag<SH>(op);
  const double* bf = a.bf + (size_t)col * a.ldf;
  const double* xpg = a.xp + (size_t)col * a.ldf;
  const double* ecg = a.ec + (size_t)col * a.ldc;
  // b and the pre-smoothed iterate of the down launch (zero outside the
  // domain in both buffers: the Dirichlet values the stencil reads)
  // (all of a thread's loads in flight before the first LDS store)
  {
    StagedN<W * H, double, kLT> hb, hu;
    StagedN<EW * EH, double, kLT> he;
    auto at = [&](const double* g, int i) {
      const int gx = R.ox + i % W, gy = R.oy + i / W;
      return ld_or_zero(g, gx >= 0 && gx < nf && gy >= 0 && gy < nf, (size_t)gy * nf + gx);
    };
    hb.load([&](int i) { return at(bf, i); });
    hu.load([&](int i) { return at(xpg, i); });
    he.load([&](int i) {
      const int I = cox + i % EW, J = coy + i / EW;
      return ld_or_zero(ecg, I >= 0 && I < nc && J >= 0 && J < nc, (size_t)J * nc + I);
    });
    hb.store(bs);
    hu.store(us[0]);
    he.store(es);
    for (int i = threadIdx.x; i < W * H; i += kLT) {
      us[1][i] = 0.0;
      ds[i] = 0.0;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < W * H; i += kLT) {
    if (R.inside(i, 0)) {
      const int gx = R.ox + i % W, gy = R.oy + i / W;
      us[0][i] += interp(es, EW, cox, coy, gx, gy);
    }
  }
  __syncthreads();
  int cur = 0;
  // post-smoothing; the last step's new values are needed on the owned nodes only
  for (int k = 0; k + 1 < kNu; ++k) {
    cheb_step<SH, W, H>(R, 1 + k, k == 0 ? 0.0 : a.sm.a[k], a.sm.c[k], inv_d, bs, us[cur],
                        us[cur ^ 1], ds, op);
    cur ^= 1;
  }
  const int x1 = (cx0 + CX >= nc) ? nf : 2 * (cx0 + CX);
  const int y1 = (cy0 + CY >= nc) ? nf : 2 * (cy0 + CY);
  const int ow = x1 - 2 * cx0, oh = y1 - 2 * cy0;
  const double ak = kNu == 1 ? 0.0 : a.sm.a[kNu - 1], ck = a.sm.c[kNu - 1];
  const double* u = us[cur];
  double* ef = a.ef + (size_t)col * a.ldf;
  double part = 0.0;
  for (int i = threadIdx.x; i < ow * oh; i += kLT) {
    const int gx = 2 * cx0 + i % ow, gy = 2 * cy0 + i / ow;
    const int q = (gy - R.oy) * W + (gx - R.ox);
    const double d = ak * ds[q] + ck * inv_d * (bs[q] - aop<SH>(u, q, W, op));
    const double e = u[q] + d;
    ef[(size_t)gy * nf + gx] = e;
    part += bs[q] * e;
  }
  if (a.part) {
    part = block_sum<kLT>(part, red);
    if (threadIdx.x == 0) a.part[(size_t)col * a.max_tiles + t] = part;
  }
}

// ---------------------------------------------------------------------------
// coarse level (n <= kMGCoarseMax): exact solve by the sine transform, four
// 64 x 64 GEMMs on the matrix cores in LDS, one work-group per column
// ---------------------------------------------------------------------------
constexpr int kE = 64;        // padded order of the exact solve
constexpr int kEL = kE + 1;   // LDS row stride (odd: no bank conflicts along columns)

struct CoarseArgs {
  int n;               // order of the coarse level (<= kMGCoarseMax)
  int64_t ld;
  const double* b;
  double* e;
  const double* dst;   // n x n sine-transform matrix S (row-major, symmetric), then l (n)
  double mu;
  double sw;           // s w of the level: the solve is with Kx + s Mx~ (see mg_vcycle)
  int nlaunch;
  int cols[kMaxCols];
  const CGScal* st;
  double* part;        // (b, e) when this is the whole V-cycle, may be null
  int max_tiles;
};

// C = A B for 64 x 64 LDS matrices (row stride kEL); with `scale`, C[y][x]
// is divided by mu (l_y + l_x) (zero outside the n x n block).  One 16 x 16
// tile per wave.
__device__ __forceinline__ void lds_gemm(const double* A, const double* B, double* C, bool scale,
                                         const double* l, double mu, double sw, int n) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int r0 = (wv & 3) * 16, c0 = (wv >> 2) * 16;
  d4 acc[4] = {};
#pragma unroll
  for (int k0 = 0; k0 < kE; k0 += 16) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      acc[j] = mfma(A[(r0 + i) * kEL + k0 + 4 * j + g], B[(k0 + 4 * j + g) * kEL + c0 + i], acc[j]);
  }
  const d4 sum = (acc[0] + acc[1]) + (acc[2] + acc[3]);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int y = r0 + 4 * q + g, x = c0 + i;
    double v = sum[q];
    if (scale)
      v = (y < n && x < n) ? v / (mu * (l[y] + l[x]) + sw * (10.0 - l[y] - l[x])) : 0.0;
    C[y * kEL + x] = v;
  }
}

__global__ __launch_bounds__(kCT) void mg_coarse_kernel(CoarseArgs a) {
  __shared__ double S[kE * kEL];
  __shared__ double X[kE * kEL];
  __shared__ double T[kE * kEL];
  __shared__ double l[kE];
  __shared__ double red[kCT / 64];
  const int col = a.cols[blockIdx.x];
  if (a.st && !a.st[col].active) return;
  const int n = a.n;
  const double* bg = a.b + (size_t)col * a.ld;
  double* eg = a.e + (size_t)col * a.ld;
  for (int i = threadIdx.x; i < kE * kE; i += kCT) {
    const int y = i / kE, x = i % kE;
    const bool in = y < n && x < n;
    S[y * kEL + x] = in ? a.dst[y * n + x] : 0.0;
    X[y * kEL + x] = in ? bg[y * n + x] : 0.0;
  }
  if (threadIdx.x < kE) l[threadIdx.x] = threadIdx.x < n ? a.dst[n * n + threadIdx.x] : 0.0;
  __syncthreads();
  lds_gemm(S, X, T, false, l, a.mu, a.sw, n);   // T = S B
  __syncthreads();
  lds_gemm(T, S, X, true, l, a.mu, a.sw, n);    // X = (T S) ./ (mu (l_y + l_x) + ...)
  __syncthreads();
  lds_gemm(S, X, T, false, l, a.mu, a.sw, n);   // T = S X
  __syncthreads();
  lds_gemm(T, S, X, false, l, a.mu, a.sw, n);   // X = T S
  __syncthreads();
  double part = 0.0;
  for (int i = threadIdx.x; i < n * n; i += kCT) {
    const double v = X[(i / n) * kEL + i % n];
    eg[i] = v;
    part += bg[i] * v;
  }
  if (a.part) {
    part = block_sum<kCT>(part, red);
    if (threadIdx.x == 0) a.part[(size_t)col * a.max_tiles] = part;
  }
}

// ---------------------------------------------------------------------------
// coarse level of order 64..kMGExactMax: the same exact solve as four
// row-major m x m GEMMs, C = A B (optionally divided by mu (l_r + l_c)), over
// many work-groups.  A work-group owns a 16 x 16 tile of C and splits the
// inner dimension (padded to kMGExactMax + 1) over its kDstWaves waves; each
// wave issues all of its loads straight from global memory (the operands are
// L2-resident) before its MFMAs, and the partial tiles are added through LDS
// in a fixed order.  Small tiles and the split give the many work-groups a
// launch of this size needs to fill the chip (5.4 us against 10 us for
// 32 x 32 tiles staged in LDS, m = 255, two columns).
// ---------------------------------------------------------------------------
constexpr int kDstWaves = 8;
constexpr int kDstK = (kMGExactMax + 1) / kDstWaves;   // inner indices per wave
static_assert(kDstK % 4 == 0, "whole MFMA steps per wave");

struct DstGemmArgs {
  int m;
  int nlaunch;
  int cols[kMaxCols];
  const double* A;     // shared (a_ld = 0) or per column
  int64_t a_ld;        // column stride of A (0: shared)
  const double* B;
  int64_t b_ld;
  double* C;
  int64_t c_ld;
  const double* l;     // eigenvalues if the product is scaled, else null
  double mu;
  double sw;
  const CGScal* st;
};

__global__ __launch_bounds__(64 * kDstWaves) void dst_gemm_kernel(DstGemmArgs a) {
  constexpr int NS = kDstK / 4;   // MFMA steps per wave
  __shared__ double red[kDstWaves - 1][256];
  const int m = a.m;
  const int nt = (m + 15) / 16;
  const int r0 = (blockIdx.x % nt) * 16, c0 = (blockIdx.x / nt) * 16;
  const int col = a.cols[blockIdx.y];
  if (a.st && !a.st[col].active) return;
  const double* A = a.A + (size_t)col * a.a_ld;
  const double* B = a.B + (size_t)col * a.b_ld;
  double* C = a.C + (size_t)col * a.c_ld;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int r = r0 + i, c = c0 + i;
  const int kb = wv * kDstK;
  double av[NS], bv[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int k = kb + 4 * s + g;
    av[s] = (r < m && k < m) ? A[(size_t)r * m + k] : 0.0;
    bv[s] = (c < m && k < m) ? B[(size_t)k * m + c] : 0.0;
  }
  // four independent accumulators: the FP64 MFMA result latency is long
  d4 acc[4] = {};
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s & 3] = mfma(av[s], bv[s], acc[s & 3]);
  const d4 sum = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  if (wv > 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) red[wv - 1][(4 * q + g) * 16 + i] = sum[q];
  }
  __syncthreads();
  if (wv != 0) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int rr = r0 + 4 * q + g;
    double v = sum[q];
#pragma unroll
    for (int w = 0; w < kDstWaves - 1; ++w) v += red[w][(4 * q + g) * 16 + i];
    if (rr < m && c < m) {
      if (a.l) v /= a.mu * (a.l[rr] + a.l[c]) + a.sw * (10.0 - a.l[rr] - a.l[c]);
      C[(size_t)rr * m + c] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// coarse level with m + 1 = L a power of two (128 or 256): the same exact
// solve, U = S [(S B S) / (mu (l_r + l_c))] S, by fast sine transforms.  The
// raw transform y_k = sum_j x_j sin(pi j k / L) of a length-m vector is, up to
// the factor -2i, the discrete Fourier transform of length N = 2L of its odd
// extension (0, x_1 .. x_m, 0, -x_m .. -x_1); the transforms of two real
// vectors x1, x2 come from one complex transform of x1 + i x2 (the transform
// of each odd real sequence is imaginary): y1 = -Im(Z) / 2, y2 = Re(Z) / 2.
// One work-group of L threads transforms two rows (or two columns) with a
// radix-2 decimation-in-time FFT in LDS, one butterfly per thread per stage.
// Three launches: rows (B S), columns (S . , the division, S .), rows (. S).
// ---------------------------------------------------------------------------
struct FstArgs {
  int m;
  int nlaunch;
  int cols[kMaxCols];
  const double* in;    // per column (stride in_ld), m x m row-major
  int64_t in_ld;
  double* out;
  int64_t out_ld;
  const double* lv;    // l_0 .. l_{m-1}
  const double* tw;    // cos, sin of pi k / L, k < L
  double mu;
  double sw;
  const CGScal* st;
};

template <int L>
__global__ __launch_bounds__(L) void fst_row_kernel(FstArgs a) {
  __shared__ double2 z[2 * L];
  __shared__ double tw[2 * L];
  const int col = a.cols[blockIdx.y];
  if (a.st && !a.st[col].active) return;
  const int m = a.m;
  const double tw0 = a.tw[threadIdx.x], tw1 = a.tw[threadIdx.x + L];   // stored with z
  const int r1 = 2 * blockIdx.x, r2 = r1 + 1;
  const double* in = a.in + (size_t)col * a.in_ld;
  double* out = a.out + (size_t)col * a.out_ld;
  fst_load<L>(
      z, m,
      [&](int j) {
        return double2{in[(size_t)r1 * m + j], r2 < m ? in[(size_t)r2 * m + j] : 0.0};
      },
      [&] {
        tw[threadIdx.x] = tw0;
        tw[threadIdx.x + L] = tw1;
      });
  fft_lds<L>(z, tw);
  const double sc = 0.5 * sqrt(2.0 / L);
  const int k = threadIdx.x + 1;   // frequency 1 .. m
  if (k <= m) {
    const double2 Z = z[k];
    out[(size_t)r1 * m + k - 1] = -Z.y * sc;
    if (r2 < m) out[(size_t)r2 * m + k - 1] = Z.x * sc;
  }
}

template <int L>
__global__ __launch_bounds__(L) void fst_col_kernel(FstArgs a) {
  __shared__ double2 z[2 * L];
  __shared__ double tw[2 * L];
  __shared__ double2 v[L];
  const int col = a.cols[blockIdx.y];
  if (a.st && !a.st[col].active) return;
  const int m = a.m;
  const double tw0 = a.tw[threadIdx.x], tw1 = a.tw[threadIdx.x + L];   // stored with z
  // a work-group reads 16 bytes of each row; the eight groups that share a
  // 128-byte line run on one XCD (consecutive block ids go round-robin over
  // the XCDs), so the line is fetched into one L2 instead of eight
  const int c1 = 2 * xcd_remap(blockIdx.x, gridDim.x), c2 = c1 + 1;
  const double* in = a.in + (size_t)col * a.in_ld;
  double* out = a.out + (size_t)col * a.out_ld;
  const int t = threadIdx.x;
  // eigenvalues of the divisor, loaded with the data (indices clamped to m - 1)
  const double lr = a.lv[min(t, m - 1)], l1 = a.lv[c1], l2 = a.lv[min(c2, m - 1)];
  fst_load<L>(
      z, m,
      [&](int j) {
        return double2{in[(size_t)j * m + c1], c2 < m ? in[(size_t)j * m + c2] : 0.0};
      },
      [&] {
        tw[threadIdx.x] = tw0;
        tw[threadIdx.x + L] = tw1;
      });
  fft_lds<L>(z, tw);
  const double sc = 0.5 * sqrt(2.0 / L);
  if (t < m) {
    // frequency t + 1 along the rows; the columns already hold frequencies c1, c2
    const double2 Z = z[t + 1];
    const double d1 = a.mu * (lr + l1) + a.sw * (10.0 - lr - l1);
    const double d2 = c2 < m ? a.mu * (lr + l2) + a.sw * (10.0 - lr - l2) : 1.0;
    v[t] = double2{-Z.y * sc / d1, c2 < m ? Z.x * sc / d2 : 0.0};
  }
  __syncthreads();
  fst_load<L>(z, m, [&](int j) { return v[j]; });
  fft_lds<L>(z, tw);
  if (t < m) {
    const double2 Z = z[t + 1];
    out[(size_t)t * m + c1] = -Z.y * sc;
    if (c2 < m) out[(size_t)t * m + c2] = Z.x * sc;
  }
}

bool fst_supported(int m) { return m + 1 == 128 || m + 1 == 256; }

// ---------------------------------------------------------------------------
// PCG launches on the finest grid (tiles TX x TY)
// ---------------------------------------------------------------------------
struct PCGArgs {
  int n;
  int64_t ld;          // stride of r, z, p, q
  int ntx, nty;
  int ncols;
  int nlaunch;
  int cols[kMaxCols];
  Op op;               // operator of the finest level
  double* x;
  int64_t ldx;
  double* r;
  const double* z;
  const double* pin;   // p of the previous iteration
  double* pout;        // p of this iteration
  double* q;
  const CGScal* prev;  // state slot written by the previous iteration
  CGScal* next;        // state slot of this iteration
  double* part_rr;     // (r, r) per fine tile (B, set-up)
  double* part_rz;     // (r, z) per level-0 up tile
  double* part_pq;     // (p, q) per fine tile (A)
  int rz_tiles;
  double* alpha;       // per column, written by B's tile 0 (0 = breakdown)
  int max_tiles;
  const double* b[kMaxCols];   // set-up only
};

// A: stopping test and beta from (r, r) and (r, z) of this work-group's
// column; p = z + beta p; q = K p; (p, q).  Tile 0 of each column writes its
// state; work-group 0 carries over the state of columns not launched.
template <bool SH>
__global__ __launch_bounds__(kT) void pcg_a_kernel(PCGArgs a) {
  constexpr int RW = TX + 2, RH = TY + 2;
  __shared__ double ps[RW * RH];
  __shared__ double red[2][kT / 64];
  const int ntiles = a.ntx * a.nty;
  const int lin = xcd_remap(blockIdx.x, a.nlaunch * ntiles);
  const int t = lin / a.nlaunch, col = a.cols[lin % a.nlaunch];
  if (blockIdx.x == 0) {
    for (int c = threadIdx.x; c < a.ncols; c += kT) {
      bool launched = false;
      for (int j = 0; j < a.nlaunch; ++j) launched |= a.cols[j] == c;
      if (!launched) a.next[c] = a.prev[c];
    }
  }
  CGScal s = a.prev[col];
  if (!s.active) {
    if (t == 0 && threadIdx.x == 0) a.next[col] = s;
    return;
  }
  // (r, r) and (r, z) in one pass over the partials
  double rr = 0.0, rz = 0.0;
  const double* prr = a.part_rr + (size_t)col * a.max_tiles;
  const double* prz = a.part_rz + (size_t)col * a.max_tiles;
  for (int u = threadIdx.x; u < ntiles; u += kT) rr += prr[u];
  for (int u = threadIdx.x; u < a.rz_tiles; u += kT) rz += prz[u];
  rr = wave_sum(rr);
  rz = wave_sum(rz);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = rr;
    red[1][threadIdx.x >> 6] = rz;
  }
  __syncthreads();
  rr = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
  rz = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  double beta;
  const bool go = pcg_decide(s, rr, rz, a.alpha[col], beta);
  if (t == 0 && threadIdx.x == 0) a.next[col] = s;
  if (!go) return;
  const int n = a.n;
  const int x0 = (t % a.ntx) * TX, y0 = (t / a.ntx) * TY;
  const double* zg = a.z + (size_t)col * a.ld;
  const double* pin = a.pin + (size_t)col * a.ld;
  double* pout = a.pout + (size_t)col * a.ld;
  double* qg = a.q + (size_t)col * a.ld;
  {
    StagedN<RW * RH, double, kT> hp;
    hp.load([&](int i) {
      const int gx = x0 - 1 + i % RW, gy = y0 - 1 + i / RW;
      const bool in = gx >= 0 && gx < n && gy >= 0 && gy < n;
      const size_t g = (size_t)gy * n + gx;
      return ld_or_zero(zg, in, g) + beta * ld_or_zero(pin, in, g);
    });
    hp.store(ps);
  }
  __syncthreads();
  double part = 0.0;
  for (int i = threadIdx.x; i < TX * TY; i += kT) {
    const int gx = x0 + i % TX, gy = y0 + i / TX;
    if (gx < n && gy < n) {
      const int qi = (i / TX + 1) * RW + (i % TX + 1);
      const double pv = ps[qi];
      const double qv = aop<SH>(ps, qi, RW, a.op);
      const size_t g = (size_t)gy * n + gx;
      pout[g] = pv;
      qg[g] = qv;
      part += pv * qv;
    }
  }
  part = block_sum<kT>(part, red[0]);
  if (threadIdx.x == 0) a.part_pq[(size_t)col * a.max_tiles + t] = part;
}

// B: alpha = rho / (p, q); x += alpha p; r -= alpha q; (r, r).
__global__ __launch_bounds__(kT) void pcg_b_kernel(PCGArgs a) {
  __shared__ double red[kT / 64];
  const int ntiles = a.ntx * a.nty;
  const int lin = xcd_remap(blockIdx.x, a.nlaunch * ntiles);
  const int t = lin / a.nlaunch, col = a.cols[lin % a.nlaunch];
  const CGScal s = a.next[col];   // written by this iteration's A
  if (!s.active) return;
  double pq = 0.0;
  const double* ppq = a.part_pq + (size_t)col * a.max_tiles;
  for (int u = threadIdx.x; u < ntiles; u += kT) pq += ppq[u];
  pq = block_sum<kT>(pq, red);
  const bool ok = pq > 0.0 && __builtin_isfinite(pq);
  const double alpha = ok ? s.rho / pq : 0.0;
  if (t == 0 && threadIdx.x == 0) a.alpha[col] = alpha;
  if (!ok) return;
  const int n = a.n;
  const int x0 = (t % a.ntx) * TX, y0 = (t / a.ntx) * TY;
  double* xg = a.x + (size_t)col * a.ldx;
  double* rg = a.r + (size_t)col * a.ld;
  const double* pg = a.pout + (size_t)col * a.ld;
  const double* qg = a.q + (size_t)col * a.ld;
  // every load of the thread's nodes before the first store (outside the
  // domain the loads read node 0 and nothing is stored)
  constexpr int NN = TX * TY / kT;
  static_assert(NN * kT == TX * TY, "whole tile nodes per thread");
  size_t g[NN];
  bool in[NN];
  double xv[NN], pv[NN], rv[NN], qv[NN];
#pragma unroll
  for (int k = 0; k < NN; ++k) {
    const int i = threadIdx.x + k * kT;
    const int gx = x0 + i % TX, gy = y0 + i / TX;
    in[k] = gx < n && gy < n;
    g[k] = in[k] ? (size_t)gy * n + gx : 0;
    xv[k] = xg[g[k]];
    pv[k] = pg[g[k]];
    rv[k] = rg[g[k]];
    qv[k] = qg[g[k]];
  }
  double part = 0.0;
#pragma unroll
  for (int k = 0; k < NN; ++k) {
    if (!in[k]) continue;
    xg[g[k]] = xv[k] + alpha * pv[k];
    const double r = rv[k] - alpha * qv[k];
    rg[g[k]] = r;
    part += r * r;
  }
  part = block_sum<kT>(part, red);
  if (threadIdx.x == 0) a.part_rr[(size_t)col * a.max_tiles + t] = part;
}

// Set-up: x = 0, r = b, both p buffers 0, partials of (b, b); both state slots
// initialised (columns in the launch list active), alpha = 1.
__global__ __launch_bounds__(kT) void pcg_setup_kernel(PCGArgs a, double rtol2, int maxit) {
  __shared__ double red[kT / 64];
  const int ntiles = a.ntx * a.nty;
  const int lin = xcd_remap(blockIdx.x, a.nlaunch * ntiles);
  const int t = lin / a.nlaunch, jb = lin % a.nlaunch, col = a.cols[jb];
  const int n = a.n;
  const int x0 = (t % a.ntx) * TX, y0 = (t / a.ntx) * TY;
  const double* bg = a.b[jb];
  double* pa = const_cast<double*>(a.pin);
  double part = 0.0;
  for (int i = threadIdx.x; i < TX * TY; i += kT) {
    const int gx = x0 + i % TX, gy = y0 + i / TX;
    if (gx < n && gy < n) {
      const size_t g = (size_t)gy * n + gx;
      const double bv = bg[g];
      a.x[g + (size_t)col * a.ldx] = 0.0;
      a.r[g + (size_t)col * a.ld] = bv;
      pa[g + (size_t)col * a.ld] = 0.0;
      a.pout[g + (size_t)col * a.ld] = 0.0;
      part += bv * bv;
    }
  }
  part = block_sum<kT>(part, red);
  if (threadIdx.x == 0) a.part_rr[(size_t)col * a.max_tiles + t] = part;
  if (blockIdx.x == 0 && threadIdx.x < kMaxCols) {
    const int c = threadIdx.x;
    bool launched = false;
    for (int j = 0; j < a.nlaunch; ++j) launched |= a.cols[j] == c;
    CGScal s{};
    s.rtol2 = rtol2;
    s.maxit = maxit;
    s.active = launched ? 1 : 0;
    a.next[c] = s;
    const_cast<CGScal*>(a.prev)[c] = s;
    a.alpha[c] = 1.0;
  }
}

int tiles_of(int n, int tx, int ty) { return ((n + tx - 1) / tx) * ((n + ty - 1) / ty); }

// Operator of level l: w_l = 4^l w_0, s w_l = 4^l sw0.
Op level_op(const MGPlan& p, int l) {
  const double swl = std::ldexp(p.sw0, 2 * l);
  return Op{p.mu, 4.0 * p.mu + 6.0 * swl, -p.mu + swl, swl};
}

PCGArgs pcg_args(const MGWork& w, int parity, const int* cols, int nlaunch, int ncols) {
  PCGArgs a{};
  a.n = w.plan.n[0];
  a.ld = w.ld[0];
  a.ntx = (a.n + TX - 1) / TX;
  a.nty = (a.n + TY - 1) / TY;
  a.ncols = ncols;
  a.nlaunch = nlaunch;
  for (int j = 0; j < nlaunch; ++j) a.cols[j] = cols[j];
  a.op = level_op(w.plan, 0);
  a.x = w.x;
  a.ldx = w.ldx;
  a.r = w.b[0];
  a.z = w.e[0];
  a.pin = w.p[parity ^ 1];
  a.pout = w.p[parity];
  a.q = w.q;
  a.prev = w.scal + (parity ^ 1) * kMaxCols;
  a.next = w.scal + parity * kMaxCols;
  a.part_rr = w.part_rr;
  a.part_rz = w.part_rz;
  a.part_pq = w.part_pq;
  a.rz_tiles = w.plan.nlev > 0 ? tiles_of(w.plan.n[1], CX, CY) : 1;
  a.alpha = w.alpha;
  a.max_tiles = w.max_tiles;
  return a;
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

bool mg_plan(const Grid& g, const Stencil& K, MGPlan* plan) {
  if (g.dim == 3) return mg3_plan(g, K, plan);
  if (g.dim != 2 || g.nx != g.ny || g.nx < 1) return false;
  // Kx must be mu times the five-point pattern (4; -1, -1, -1, -1)
  const double c0 = K.c[13];
  if (!(c0 > 0.0)) return false;
  const double mu = c0 / 4.0;
  for (int i = 0; i < 27; ++i) {
    double want = 0.0;
    if (i == 13) want = c0;
    if (i == 12 || i == 14 || i == 10 || i == 16) want = -mu;
    if (K.c[i] != want) return false;
  }
  MGPlan p{};
  p.dim = 2;
  p.mu = mu;
  int L = 0, n = g.nx;
  p.n[0] = n;
  // halve while above kMGExactMax, and at least once above kMGCoarseMax, so
  // that every grid larger than kMGCoarseMax keeps a smoothed fine level
  while (n > kMGExactMax || (L == 0 && n > kMGCoarseMax)) {
    if ((n & 1) == 0 || L + 1 >= kMGMaxLevels) return false;   // does not halve
    n = (n - 1) / 2;
    p.n[++L] = n;
  }
  p.nlev = L;
  p.exact = n;
  *plan = p;
  return true;
}

int mg_max_tiles(const MGPlan& p) {
  if (p.dim == 3) return mg3_max_tiles(p);
  int t = tiles_of(p.n[0], TX, TY);
  if (p.nlev > 0) t = std::max(t, tiles_of(p.n[1], CX, CY));
  return std::max(t, 1);
}

void mg_dst_table(int m, double* out) {
  // S[y][x] = sqrt(2 / (m + 1)) sin(pi (y + 1)(x + 1) / (m + 1)); l_y = 2 - 2 cos(pi (y + 1) / (m + 1));
  // then cos, sin of pi k / (m + 1), k <= m (the twiddles of the fast transform)
  const double pi = 3.14159265358979323846;
  const double s = std::sqrt(2.0 / (m + 1));
  for (int y = 0; y < m; ++y)
    for (int x = 0; x < m; ++x) {
      // reduce the angle's integer multiple modulo 2 (m + 1) before the sine
      const long long num = (long long)(y + 1) * (x + 1) % (2LL * (m + 1));
      out[y * m + x] = s * std::sin(pi * (double)num / (m + 1));
    }
  for (int y = 0; y < m; ++y) out[m * m + y] = 2.0 - 2.0 * std::cos(pi * (y + 1) / (m + 1));
  double* tw = out + (size_t)m * (m + 1);
  for (int k = 0; k <= m; ++k) {
    tw[2 * k] = std::cos(pi * k / (m + 1));
    tw[2 * k + 1] = std::sin(pi * k / (m + 1));
  }
}

size_t mg_dst_table_size(int m) { return (size_t)m * (m + 1) + 2 * (size_t)(m + 1); }

void mg_vcycle(const MGWork& w, const CGScal* act, const int* cols, int nlaunch, bool partials,
               hipStream_t st) {
  if (w.plan.dim == 3) return mg3_vcycle(w, act, cols, nlaunch, partials, st);
  const MGPlan& p = w.plan;
  const int L = p.nlev;
  const Smooth sm = smooth_coefficients(0.5);   // [1/2, 2]: the oscillatory part in 2-D
  const bool sh = p.sw0 != 0.0;
  // the coarsest level's s w: its exact sine-transform solve takes the mass
  // part without the SW-NE coupling, s w (6; 1 x 4), which the transform
  // diagonalises (symbol s w (10 - l_r - l_c)); with s = 0 it is exact
  const double swL = std::ldexp(p.sw0, 2 * L);
  for (int l = 0; l < L; ++l) {
    LevelArgs a{};
    a.nf = p.n[l];
    a.nc = p.n[l + 1];
    a.ldf = w.ld[l];
    a.ldc = w.ld[l + 1];
    a.bf = w.b[l];
    a.bc = w.b[l + 1];
    a.xp = w.xp[l];
    a.ntx = (a.nc + CX - 1) / CX;
    a.nty = (a.nc + CY - 1) / CY;
    a.nlaunch = nlaunch;
    for (int j = 0; j < nlaunch; ++j) a.cols[j] = cols[j];
    a.st = act;
    a.op = level_op(p, l);
    a.sm = sm;
    const double by = 8.0 * (2.0 * a.nf * a.nf + (double)a.nc * a.nc) * nlaunch;
    if (sh)
      launch(STS_K_MG_DOWN, by, mg_down_kernel<true>, dim3(a.ntx * a.nty * nlaunch), dim3(kLT), 0,
             st, a);
    else
      launch(STS_K_MG_DOWN, by, mg_down_kernel<false>, dim3(a.ntx * a.nty * nlaunch), dim3(kLT), 0,
             st, a);
    STS_HIP(hipGetLastError());
  }
  if (p.n[L] <= kMGCoarseMax) {
    CoarseArgs c{};
    c.n = p.n[L];
    c.ld = w.ld[L];
    c.b = w.b[L];
    c.e = w.e[L];
    c.dst = w.dst;
    c.mu = p.mu;
    c.sw = swL;
    c.nlaunch = nlaunch;
    for (int j = 0; j < nlaunch; ++j) c.cols[j] = cols[j];
    c.st = act;
    c.part = (partials && L == 0) ? w.part_rz : nullptr;
    c.max_tiles = w.max_tiles;
    launch(STS_K_MG_COARSE, 16.0 * c.n * c.n * nlaunch, mg_coarse_kernel, dim3(nlaunch), dim3(kCT),
           0, st, c);
  } else if (fst_supported(p.n[L])) {
    // e_L = S (S b_L S ./ (mu (l_r + l_c))) S by fast sine transforms
    const int m = p.n[L];
    FstArgs f{};
    f.m = m;
    f.nlaunch = nlaunch;
    for (int j = 0; j < nlaunch; ++j) f.cols[j] = cols[j];
    f.lv = w.dst + (size_t)m * m;
    f.tw = w.dst + (size_t)m * (m + 1);
    f.mu = p.mu;
    f.sw = swL;
    f.st = act;
    const int64_t ld = w.ld[L];
    const dim3 grid((m + 1) / 2, nlaunch);
    const double by = 16.0 * (double)m * m * nlaunch;   // read and write one m x m array
    auto stage = [&](int kind, const double* in, double* out) {
      f.in = in;
      f.in_ld = ld;
      f.out = out;
      f.out_ld = ld;
      if (m + 1 == 256) {
        if (kind == 0) launch(STS_K_MG_COARSE, by, fst_row_kernel<256>, grid, dim3(256), 0, st, f);
        else launch(STS_K_MG_COARSE, by, fst_col_kernel<256>, grid, dim3(256), 0, st, f);
      } else {
        if (kind == 0) launch(STS_K_MG_COARSE, by, fst_row_kernel<128>, grid, dim3(128), 0, st, f);
        else launch(STS_K_MG_COARSE, by, fst_col_kernel<128>, grid, dim3(128), 0, st, f);
      }
      STS_HIP(hipGetLastError());
    };
    stage(0, w.b[L], w.t1);      // T = B S (rows)
    stage(1, w.t1, w.t2);        // X = S (S T ./ D) (columns)
    stage(0, w.t2, w.e[L]);      // e = X S (rows)
  } else {
    // e_L = S (S b_L S ./ (mu (l_r + l_c))) S, four GEMMs (L >= 1 here)
    const int m = p.n[L];
    const double* S = w.dst;
    const double* lv = w.dst + (size_t)m * m;
    DstGemmArgs g{};
    g.m = m;
    g.nlaunch = nlaunch;
    for (int j = 0; j < nlaunch; ++j) g.cols[j] = cols[j];
    g.mu = p.mu;
    g.sw = swL;
    g.st = act;
    const int nt = (m + 15) / 16;
    const dim3 grid(nt * nt, nlaunch);
    const double by = 8.0 * 3.0 * (double)m * m * nlaunch;
    auto gemm = [&](const double* A, int64_t ald, const double* B, int64_t bld, double* C,
                    int64_t cld, const double* l) {
      g.A = A;
      g.a_ld = ald;
      g.B = B;
      g.b_ld = bld;
      g.C = C;
      g.c_ld = cld;
      g.l = l;
      launch(STS_K_MG_COARSE, by, dst_gemm_kernel, grid, dim3(64 * kDstWaves), 0, st, g);
    };
    const int64_t ld = w.ld[L];
    gemm(S, 0, w.b[L], ld, w.t1, ld, nullptr);    // T = S B
    gemm(w.t1, ld, S, 0, w.t2, ld, lv);           // X = (T S) ./ (mu (l_r + l_c))
    gemm(S, 0, w.t2, ld, w.t1, ld, nullptr);      // T = S X
    gemm(w.t1, ld, S, 0, w.e[L], ld, nullptr);    // e = T S
  }
  for (int l = L - 1; l >= 0; --l) {
    LevelArgs a{};
    a.nf = p.n[l];
    a.nc = p.n[l + 1];
    a.ldf = w.ld[l];
    a.ldc = w.ld[l + 1];
    a.bf = w.b[l];
    a.ec = w.e[l + 1];
    a.ef = w.e[l];
    a.xp = w.xp[l];
    a.ntx = (a.nc + CX - 1) / CX;
    a.nty = (a.nc + CY - 1) / CY;
    a.nlaunch = nlaunch;
    for (int j = 0; j < nlaunch; ++j) a.cols[j] = cols[j];
    a.st = act;
    a.op = level_op(p, l);
    a.sm = sm;
    a.part = (partials && l == 0) ? w.part_rz : nullptr;
    a.max_tiles = w.max_tiles;
    const double by = 8.0 * (3.0 * a.nf * a.nf + (double)a.nc * a.nc) * nlaunch;
    if (sh)
      launch(STS_K_MG_UP, by, mg_up_kernel<true>, dim3(a.ntx * a.nty * nlaunch), dim3(kLT), 0, st,
             a);
    else
      launch(STS_K_MG_UP, by, mg_up_kernel<false>, dim3(a.ntx * a.nty * nlaunch), dim3(kLT), 0, st,
             a);
    STS_HIP(hipGetLastError());
  }
}

void pcg_setup(const MGWork& w, const double* const* b, const int* cols, int nlaunch, int ncols,
               double rtol, int maxit, hipStream_t st) {
  if (w.plan.dim == 3) return pcg3_setup(w, b, cols, nlaunch, ncols, rtol, maxit, st);
  // state slot 0 is "previous" for the first iteration (parity 1)
  PCGArgs a = pcg_args(w, 0, cols, nlaunch, ncols);
  for (int j = 0; j < nlaunch; ++j) a.b[j] = b[j];
  pcg_setup_kernel<<<a.ntx * a.nty * nlaunch, kT, 0, st>>>(a, rtol * rtol, maxit);
  STS_HIP(hipGetLastError());
}

void pcg_iterate(const MGWork& w, int parity, const int* cols, int nlaunch, int ncols,
                 hipStream_t st) {
  if (w.plan.dim == 3) return pcg3_iterate(w, parity, cols, nlaunch, ncols, st);
  mg_vcycle(w, w.scal + (parity ^ 1) * kMaxCols, cols, nlaunch, true, st);
  const PCGArgs a = pcg_args(w, parity, cols, nlaunch, ncols);
  const int blocks = a.ntx * a.nty * nlaunch;
  const double nn = (double)a.n * a.n * nlaunch;
  if (w.plan.sw0 != 0.0)
    launch(STS_K_PCG_A, 32.0 * nn, pcg_a_kernel<true>, dim3(blocks), dim3(kT), 0, st, a);
  else
    launch(STS_K_PCG_A, 32.0 * nn, pcg_a_kernel<false>, dim3(blocks), dim3(kT), 0, st, a);
  STS_HIP(hipGetLastError());
  launch(STS_K_PCG_B, 48.0 * nn, pcg_b_kernel, dim3(blocks), dim3(kT), 0, st, a);
  STS_HIP(hipGetLastError());
}

}  // namespace sts
