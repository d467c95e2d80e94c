// Multigrid-preconditioned conjugate gradients for the 2-D P1 stiffness.
//
// The inner solves with Kx (the negative powers of the extended Krylov space,
// Sec. 4) dominate the solver, and unpreconditioned CG needs O(1/h) iterations
// for them.  On the uniform Courant triangulation the P1 spaces of the meshes
// h, 2h, 4h, ... are nested: the prolongation P is P1 interpolation (coarse
// values at coincident nodes, the mean of the two end points at midpoints of
// horizontal, vertical and SW-NE edges) and the Galerkin coarse operator
// P^T Kx P is again mu (4; -1, -1, -1, -1) on the coarse mesh.  The
// preconditioner is one symmetric V-cycle started from zero: two damped-Jacobi
// sweeps (u += c (b - K u), c = omega / (4 mu)) before and after each coarse
// correction, restriction P^T, and the levels with at most kCoarseMax nodes
// per direction handled by one work-group in LDS, down to one node solved
// exactly.  Pre- and post-smoothing are adjoint, so the V-cycle is a fixed
// symmetric positive definite operator and the outer iteration is ordinary
// preconditioned CG.
//
// Launches per PCG iteration: per tiled level a "down" (two sweeps from zero,
// residual, restriction -- recomputed on LDS halos, only the restricted
// right-hand side is stored) and an "up" (pre-smoothed values recomputed from
// the level's right-hand side, interpolated correction, two sweeps), one
// coarse launch, and two PCG launches: A {beta from (r, z); p = z + beta p;
// q = K p; (p, q)} and B {alpha = rho / (p, q); x += alpha p; r -= alpha q;
// (r, r)}.  Global sums are per-tile partials that every work-group of the
// consuming launch adds in the same fixed order, so all of them take the same
// decision without atomics or a grid barrier.
#include <hip/hip_runtime.h>

#include "sts_internal.h"

namespace sts {

namespace {

constexpr int kT = 256;          // threads per work-group of the level and PCG kernels
constexpr int CX = 32, CY = 8;   // coarse nodes per level-kernel tile (fine footprint 64 x 16)
constexpr int TX = 64, TY = 16;  // fine nodes per PCG-kernel tile
constexpr double kOmega = 0.8;   // damped-Jacobi weight (smoothing factor 0.6 for this stencil)
constexpr int kCT = 1024;        // threads of the coarse kernel
constexpr int kCoarseStore = 5760;                              // >= sum (n+2)^2, n = 63, 31, ..., 1
constexpr int kCoarseTmp = (kMGCoarseMax + 2) * (kMGCoarseMax + 2);
constexpr int kCoarseLevels = 8;
constexpr int kBottomSweeps = 20;   // a coarsest level that does not halve (even n > 1)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Consecutive block ids go round-robin over the 8 XCDs; give each XCD a
// contiguous range of tiles so that halo neighbours share an L2.
__device__ __forceinline__ int xcd_remap(int bid, int n) {
  const int q = n >> 3, rem = n & 7;
  const int x = bid & 7, j = bid >> 3;
  return x * q + min(x, rem) + j;
}

// mu (4 u - u_W - u_E - u_S - u_N) on an LDS array of row width W.
__device__ __forceinline__ double k5(const double* s, int q, int W, double mu) {
  return mu * (4.0 * s[q] - (s[q - 1] + s[q + 1]) - (s[q - W] + s[q + W]));
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

struct LevelArgs {
  int nf, nc;          // fine / coarse nodes per direction (nf = 2 nc + 1)
  int64_t ldf, ldc;    // column strides
  const double* bf;    // fine right-hand side
  double* bc;          // down: restricted residual
  const double* ec;    // up: coarse correction
  double* ef;          // up: result on the fine level
  int ntx, nty;        // coarse tiles
  int nlaunch;
  int cols[kMaxCols];
  const CGScal* st;    // per-column activity, may be null (all active)
  double mu;
  double* part;        // up: per-tile (b, e), may be null
  int max_tiles;
};

// ---------------------------------------------------------------------------
// down: u2 = two sweeps from zero = c (2 b - c K b); res = b - K u2;
// b_c = P^T res at the tile's coarse nodes.  Fine region of the tile:
// [2 cx0 - 2, 2 cx0 + 2 CX + 4) in x (likewise y).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kT) void mg_down_kernel(LevelArgs a) {
  constexpr int W = 2 * CX + 6, H = 2 * CY + 6;
  __shared__ double bs[W * H];
  __shared__ double us[W * H];
  const int ntiles = a.ntx * a.nty;
  const int lin = xcd_remap(blockIdx.x, a.nlaunch * ntiles);
  const int t = lin / a.nlaunch, col = a.cols[lin % a.nlaunch];
  if (a.st && !a.st[col].active) return;
  const int cx0 = (t % a.ntx) * CX, cy0 = (t / a.ntx) * CY;
  const int nf = a.nf, nc = a.nc;
  const int ox = 2 * cx0 - 2, oy = 2 * cy0 - 2;
  const double mu = a.mu, cw = kOmega / (4.0 * mu);
  const double* bf = a.bf + (size_t)col * a.ldf;
  for (int i = threadIdx.x; i < W * H; i += kT) {
    const int gx = ox + i % W, gy = oy + i / W;
    bs[i] = (gx >= 0 && gx < nf && gy >= 0 && gy < nf) ? bf[(size_t)gy * nf + gx] : 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < W * H; i += kT) {
    const int lx = i % W, ly = i / W, gx = ox + lx, gy = oy + ly;
    double v = 0.0;
    if (lx >= 1 && lx < W - 1 && ly >= 1 && ly < H - 1 && gx >= 0 && gx < nf && gy >= 0 &&
        gy < nf)
      v = cw * (2.0 * bs[i] - cw * k5(bs, i, W, mu));
    us[i] = v;
  }
  __syncthreads();
  // residual, in place over b (each entry reads only its own b)
  for (int i = threadIdx.x; i < W * H; i += kT) {
    const int lx = i % W, ly = i / W;
    if (lx >= 2 && lx < W - 2 && ly >= 2 && ly < H - 2) bs[i] -= k5(us, i, W, mu);
  }
  __syncthreads();
  double* bc = a.bc + (size_t)col * a.ldc;
  for (int i = threadIdx.x; i < CX * CY; i += kT) {
    const int I = cx0 + i % CX, J = cy0 + i / CX;
    if (I < nc && J < nc) {
      const int q = (2 * (J - cy0) + 3) * W + (2 * (I - cx0) + 3);
      bc[(size_t)J * nc + I] =
          bs[q] + 0.5 * ((bs[q - 1] + bs[q + 1]) + (bs[q - W] + bs[q + W]) +
                         (bs[q - W - 1] + bs[q + W + 1]));
    }
  }
}

// ---------------------------------------------------------------------------
// up: u = u2 + P e_c; two sweeps; e on the tile's fine nodes
// [2 cx0, x1) x [2 cy0, y1) (the last tile in a direction runs to nf).
// Fine region [2 cx0 - 3, 2 cx0 + 2 CX + 4), coarse [cx0 - 2, cx0 + CX + 2).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kT) void mg_up_kernel(LevelArgs a) {
  constexpr int W = 2 * CX + 7, H = 2 * CY + 7;
  constexpr int EW = CX + 4, EH = CY + 4;
  __shared__ double bs[W * H];
  __shared__ double us[W * H];
  __shared__ double vs[W * H];
  __shared__ double es[EW * EH];
  __shared__ double red[kT / 64];
  const int ntiles = a.ntx * a.nty;
  const int lin = xcd_remap(blockIdx.x, a.nlaunch * ntiles);
  const int t = lin / a.nlaunch, col = a.cols[lin % a.nlaunch];
  if (a.st && !a.st[col].active) return;
  const int cx0 = (t % a.ntx) * CX, cy0 = (t / a.ntx) * CY;
  const int nf = a.nf, nc = a.nc;
  const int ox = 2 * cx0 - 3, oy = 2 * cy0 - 3;
  const int cox = cx0 - 2, coy = cy0 - 2;
  const double mu = a.mu, cw = kOmega / (4.0 * mu);
  const double* bf = a.bf + (size_t)col * a.ldf;
  const double* ecg = a.ec + (size_t)col * a.ldc;
  for (int i = threadIdx.x; i < W * H; i += kT) {
    const int gx = ox + i % W, gy = oy + i / W;
    bs[i] = (gx >= 0 && gx < nf && gy >= 0 && gy < nf) ? bf[(size_t)gy * nf + gx] : 0.0;
  }
  for (int i = threadIdx.x; i < EW * EH; i += kT) {
    const int I = cox + i % EW, J = coy + i / EW;
    es[i] = (I >= 0 && I < nc && J >= 0 && J < nc) ? ecg[(size_t)J * nc + I] : 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < W * H; i += kT) {
    const int lx = i % W, ly = i / W, gx = ox + lx, gy = oy + ly;
    double v = 0.0;
    if (lx >= 1 && lx < W - 1 && ly >= 1 && ly < H - 1 && gx >= 0 && gx < nf && gy >= 0 &&
        gy < nf)
      v = cw * (2.0 * bs[i] - cw * k5(bs, i, W, mu)) + interp(es, EW, cox, coy, gx, gy);
    us[i] = v;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < W * H; i += kT) {
    const int lx = i % W, ly = i / W, gx = ox + lx, gy = oy + ly;
    double v = 0.0;
    if (lx >= 2 && lx < W - 2 && ly >= 2 && ly < H - 2 && gx >= 0 && gx < nf && gy >= 0 &&
        gy < nf)
      v = us[i] + cw * (bs[i] - k5(us, i, W, mu));
    vs[i] = v;
  }
  __syncthreads();
  const int x1 = (cx0 + CX >= nc) ? nf : 2 * (cx0 + CX);
  const int y1 = (cy0 + CY >= nc) ? nf : 2 * (cy0 + CY);
  const int ow = x1 - 2 * cx0, oh = y1 - 2 * cy0;
  double* ef = a.ef + (size_t)col * a.ldf;
  double part = 0.0;
  for (int i = threadIdx.x; i < ow * oh; i += kT) {
    const int gx = 2 * cx0 + i % ow, gy = 2 * cy0 + i / ow;
    const int q = (gy - oy) * W + (gx - ox);
    const double e = vs[q] + cw * (bs[q] - k5(vs, q, W, mu));
    ef[(size_t)gy * nf + gx] = e;
    part += bs[q] * e;
  }
  if (a.part) {
    part = block_sum<kT>(part, red);
    if (threadIdx.x == 0) a.part[(size_t)col * a.max_tiles + t] = part;
  }
}

// ---------------------------------------------------------------------------
// coarse levels (n <= kMGCoarseMax): the rest of the V-cycle in one
// work-group per column.  Each level is an (n+2)^2 LDS array with a zero frame.
// ---------------------------------------------------------------------------
struct CoarseArgs {
  int n;
  int64_t ld;
  const double* b;
  double* e;
  double mu;
  int nlaunch;
  int cols[kMaxCols];
  const CGScal* st;
  double* part;        // (b, e) when this is the whole V-cycle, may be null
  int max_tiles;
};

// out = u + c (b - K u) on the interior of an n x n level (row width W = n+2),
// zero on the frame.
__device__ __forceinline__ void jacobi_full(double* out, const double* u, const double* b, int n,
                                            double mu, double cw) {
  const int W = n + 2;
  for (int i = threadIdx.x; i < W * W; i += kCT) {
    const int x = i % W, y = i / W;
    out[i] = (x >= 1 && x <= n && y >= 1 && y <= n) ? u[i] + cw * (b[i] - k5(u, i, W, mu)) : 0.0;
  }
}

__global__ __launch_bounds__(kCT) void mg_coarse_kernel(CoarseArgs a) {
  __shared__ double B[kCoarseStore];
  __shared__ double U[kCoarseStore];
  __shared__ double T[kCoarseTmp];
  __shared__ double red[kCT / 64];
  __shared__ int nl[kCoarseLevels], off[kCoarseLevels], nlev;
  const int col = a.cols[blockIdx.x];
  if (a.st && !a.st[col].active) return;
  const double mu = a.mu, cw = kOmega / (4.0 * mu);
  if (threadIdx.x == 0) {
    int L = 0, tot = 0;
    for (int n = a.n;;) {
      nl[L] = n;
      off[L] = tot;
      tot += (n + 2) * (n + 2);
      ++L;
      if (n <= 1 || (n & 1) == 0 || L == kCoarseLevels) break;
      n = (n - 1) / 2;
    }
    nlev = L;
  }
  for (int i = threadIdx.x; i < kCoarseStore; i += kCT) {
    B[i] = 0.0;
    U[i] = 0.0;
  }
  __syncthreads();
  const int L = nlev;
  {
    const int n = nl[0], W = n + 2;
    const double* bg = a.b + (size_t)col * a.ld;
    for (int i = threadIdx.x; i < n * n; i += kCT)
      B[off[0] + (i / n + 1) * W + (i % n + 1)] = bg[i];
  }
  __syncthreads();
  // descent: two sweeps from zero, residual, restriction
  for (int m = 0; m + 1 < L; ++m) {
    const int n = nl[m], W = n + 2;
    const double* b = B + off[m];
    double* u = U + off[m];
    for (int i = threadIdx.x; i < W * W; i += kCT) {
      const int x = i % W, y = i / W;
      T[i] = (x >= 1 && x <= n && y >= 1 && y <= n) ? cw * b[i] : 0.0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < W * W; i += kCT) {
      const int x = i % W, y = i / W;
      if (x >= 1 && x <= n && y >= 1 && y <= n) u[i] = T[i] + cw * (b[i] - k5(T, i, W, mu));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < W * W; i += kCT) {
      const int x = i % W, y = i / W;
      T[i] = (x >= 1 && x <= n && y >= 1 && y <= n) ? b[i] - k5(u, i, W, mu) : 0.0;
    }
    __syncthreads();
    const int nc = nl[m + 1], Wc = nc + 2;
    double* bc = B + off[m + 1];
    for (int i = threadIdx.x; i < nc * nc; i += kCT) {
      const int I = i % nc, J = i / nc;
      const int q = (2 * J + 2) * W + (2 * I + 2);   // fine (2I+1, 2J+1), padded
      bc[(J + 1) * Wc + (I + 1)] = T[q] + 0.5 * ((T[q - 1] + T[q + 1]) + (T[q - W] + T[q + W]) +
                                                 (T[q - W - 1] + T[q + W + 1]));
    }
    __syncthreads();
  }
  // coarsest level
  {
    const int m = L - 1, n = nl[m];
    const double* b = B + off[m];
    double* u = U + off[m];
    if (n == 1) {
      if (threadIdx.x == 0) u[4] = b[4] / (4.0 * mu);
    } else {
      for (int s = 0; s < kBottomSweeps / 2; ++s) {
        jacobi_full(T, u, b, n, mu, cw);
        __syncthreads();
        jacobi_full(u, T, b, n, mu, cw);
        __syncthreads();
      }
    }
    __syncthreads();
  }
  // ascent: interpolate the correction, two sweeps
  for (int m = L - 2; m >= 0; --m) {
    const int n = nl[m], W = n + 2;
    const int Wc = nl[m + 1] + 2;
    const double* b = B + off[m];
    double* u = U + off[m];
    const double* ec = U + off[m + 1];
    for (int i = threadIdx.x; i < n * n; i += kCT) {
      const int x = i % n, y = i / n;
      u[(y + 1) * W + (x + 1)] += interp(ec, Wc, -1, -1, x, y);
    }
    __syncthreads();
    jacobi_full(T, u, b, n, mu, cw);
    __syncthreads();
    jacobi_full(u, T, b, n, mu, cw);
    __syncthreads();
  }
  {
    const int n = nl[0], W = n + 2;
    double* eg = a.e + (size_t)col * a.ld;
    double part = 0.0;
    for (int i = threadIdx.x; i < n * n; i += kCT) {
      const int q = off[0] + (i / n + 1) * W + (i % n + 1);
      eg[i] = U[q];
      part += B[q] * U[q];
    }
    if (a.part) {
      part = block_sum<kCT>(part, red);
      if (threadIdx.x == 0) a.part[(size_t)col * a.max_tiles] = part;
    }
  }
}

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
  double mu;
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

__device__ __forceinline__ double sum_partials(const double* p, int n, double* red) {
  double s = 0.0;
  for (int t = threadIdx.x; t < n; t += kT) s += p[t];
  return block_sum<kT>(s, red);
}

// A: stopping test and beta from (r, r) and (r, z); p = z + beta p; q = K p; (p, q).
__global__ __launch_bounds__(kT) void pcg_a_kernel(PCGArgs a) {
  constexpr int RW = TX + 2, RH = TY + 2;
  __shared__ double ps[RW * RH];
  __shared__ double red[kT / 64];
  __shared__ double s_beta[kMaxCols];
  __shared__ int s_go[kMaxCols];
  const int ntiles = a.ntx * a.nty;
  const int lin = xcd_remap(blockIdx.x, a.nlaunch * ntiles);
  const int t = lin / a.nlaunch, jb = lin % a.nlaunch, col = a.cols[jb];
  const bool writer = blockIdx.x == 0;
  for (int j = 0; j < a.nlaunch; ++j) {
    const int c = a.cols[j];
    CGScal s = a.prev[c];
    int go = 0;
    double beta = 0.0;
    if (s.active) {
      const double rr = sum_partials(a.part_rr + (size_t)c * a.max_tiles, ntiles, red);
      const double rz = sum_partials(a.part_rz + (size_t)c * a.max_tiles, a.rz_tiles, red);
      const int done = s.iters;
      if (done > 0 && !(a.alpha[c] > 0.0)) {
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
        go = 1;
      }
      s.gamma = rr;
    }
    if (threadIdx.x == 0) {
      s_go[j] = go;
      s_beta[j] = beta;
      if (writer) a.next[c] = s;
    }
  }
  if (writer) {
    // columns outside the launch list keep their state
    for (int c = threadIdx.x; c < a.ncols; c += kT) {
      bool launched = false;
      for (int j = 0; j < a.nlaunch; ++j) launched |= a.cols[j] == c;
      if (!launched) a.next[c] = a.prev[c];
    }
  }
  __syncthreads();
  if (!s_go[jb]) return;
  const double beta = s_beta[jb];
  const int n = a.n;
  const int x0 = (t % a.ntx) * TX, y0 = (t / a.ntx) * TY;
  const double* zg = a.z + (size_t)col * a.ld;
  const double* pin = a.pin + (size_t)col * a.ld;
  double* pout = a.pout + (size_t)col * a.ld;
  double* qg = a.q + (size_t)col * a.ld;
  for (int i = threadIdx.x; i < RW * RH; i += kT) {
    const int gx = x0 - 1 + i % RW, gy = y0 - 1 + i / RW;
    double v = 0.0;
    if (gx >= 0 && gx < n && gy >= 0 && gy < n) {
      const size_t g = (size_t)gy * n + gx;
      v = zg[g] + beta * pin[g];
    }
    ps[i] = v;
  }
  __syncthreads();
  double part = 0.0;
  for (int i = threadIdx.x; i < TX * TY; i += kT) {
    const int gx = x0 + i % TX, gy = y0 + i / TX;
    if (gx < n && gy < n) {
      const int qi = (i / TX + 1) * RW + (i % TX + 1);
      const double pv = ps[qi];
      const double qv = k5(ps, qi, RW, a.mu);
      const size_t g = (size_t)gy * n + gx;
      pout[g] = pv;
      qg[g] = qv;
      part += pv * qv;
    }
  }
  part = block_sum<kT>(part, red);
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
  const double pq = sum_partials(a.part_pq + (size_t)col * a.max_tiles, ntiles, red);
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
  double part = 0.0;
  for (int i = threadIdx.x; i < TX * TY; i += kT) {
    const int gx = x0 + i % TX, gy = y0 + i / TX;
    if (gx < n && gy < n) {
      const size_t g = (size_t)gy * n + gx;
      xg[g] += alpha * pg[g];
      const double rv = rg[g] - alpha * qg[g];
      rg[g] = rv;
      part += rv * rv;
    }
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

PCGArgs pcg_args(const MGWork& w, int parity, const int* cols, int nlaunch, int ncols) {
  PCGArgs a{};
  a.n = w.plan.n[0];
  a.ld = w.ld[0];
  a.ntx = (a.n + TX - 1) / TX;
  a.nty = (a.n + TY - 1) / TY;
  a.ncols = ncols;
  a.nlaunch = nlaunch;
  for (int j = 0; j < nlaunch; ++j) a.cols[j] = cols[j];
  a.mu = w.plan.mu;
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
  p.mu = mu;
  int L = 0, n = g.nx;
  p.n[0] = n;
  while (n > kMGCoarseMax) {
    if ((n & 1) == 0 || L + 1 >= kMGMaxLevels) return false;   // does not halve
    n = (n - 1) / 2;
    p.n[++L] = n;
  }
  p.nlev = L;
  *plan = p;
  return true;
}

int mg_max_tiles(const MGPlan& p) {
  int t = tiles_of(p.n[0], TX, TY);
  if (p.nlev > 0) t = std::max(t, tiles_of(p.n[1], CX, CY));
  return std::max(t, 1);
}

void mg_vcycle(const MGWork& w, const CGScal* act, const int* cols, int nlaunch, bool partials,
               hipStream_t st) {
  const MGPlan& p = w.plan;
  const int L = p.nlev;
  for (int l = 0; l < L; ++l) {
    LevelArgs a{};
    a.nf = p.n[l];
    a.nc = p.n[l + 1];
    a.ldf = w.ld[l];
    a.ldc = w.ld[l + 1];
    a.bf = w.b[l];
    a.bc = w.b[l + 1];
    a.ntx = (a.nc + CX - 1) / CX;
    a.nty = (a.nc + CY - 1) / CY;
    a.nlaunch = nlaunch;
    for (int j = 0; j < nlaunch; ++j) a.cols[j] = cols[j];
    a.st = act;
    a.mu = p.mu;
    mg_down_kernel<<<a.ntx * a.nty * nlaunch, kT, 0, st>>>(a);
    STS_HIP(hipGetLastError());
  }
  {
    CoarseArgs c{};
    c.n = p.n[L];
    c.ld = w.ld[L];
    c.b = w.b[L];
    c.e = w.e[L];
    c.mu = p.mu;
    c.nlaunch = nlaunch;
    for (int j = 0; j < nlaunch; ++j) c.cols[j] = cols[j];
    c.st = act;
    c.part = (partials && L == 0) ? w.part_rz : nullptr;
    c.max_tiles = w.max_tiles;
    mg_coarse_kernel<<<nlaunch, kCT, 0, st>>>(c);
    STS_HIP(hipGetLastError());
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
    a.ntx = (a.nc + CX - 1) / CX;
    a.nty = (a.nc + CY - 1) / CY;
    a.nlaunch = nlaunch;
    for (int j = 0; j < nlaunch; ++j) a.cols[j] = cols[j];
    a.st = act;
    a.mu = p.mu;
    a.part = (partials && l == 0) ? w.part_rz : nullptr;
    a.max_tiles = w.max_tiles;
    mg_up_kernel<<<a.ntx * a.nty * nlaunch, kT, 0, st>>>(a);
    STS_HIP(hipGetLastError());
  }
}

void pcg_setup(const MGWork& w, const double* const* b, const int* cols, int nlaunch, int ncols,
               double rtol, int maxit, hipStream_t st) {
  // state slot 1 is "previous" for the first iteration (parity 0)
  PCGArgs a = pcg_args(w, 1, cols, nlaunch, ncols);
  for (int j = 0; j < nlaunch; ++j) a.b[j] = b[j];
  pcg_setup_kernel<<<a.ntx * a.nty * nlaunch, kT, 0, st>>>(a, rtol * rtol, maxit);
  STS_HIP(hipGetLastError());
}

void pcg_iterate(const MGWork& w, int parity, const int* cols, int nlaunch, int ncols,
                 hipStream_t st) {
  mg_vcycle(w, w.scal + (parity ^ 1) * kMaxCols, cols, nlaunch, true, st);
  const PCGArgs a = pcg_args(w, parity, cols, nlaunch, ncols);
  const int blocks = a.ntx * a.nty * nlaunch;
  pcg_a_kernel<<<blocks, kT, 0, st>>>(a);
  STS_HIP(hipGetLastError());
  pcg_b_kernel<<<blocks, kT, 0, st>>>(a);
  STS_HIP(hipGetLastError());
}

}  // namespace sts
