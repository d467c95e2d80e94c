// Multigrid-preconditioned conjugate gradients for the 3-D 7-point stiffness.
//
// Kx = c (6; -1 x 6), c = mu h, is the P1 stiffness of the Kuhn triangulation
// of the uniform grid (every cube cut into six tetrahedra around its x+y+z
// diagonal).  The paper's 3-D heat problem (Sec. 5, Example 1) uses linear
// elements; pairing this 7-point stiffness with the consistent trilinear (Q1)
// mass is this library's reading of a trilinear-mass / 7-point-stiffness
// discretisation, which the paper itself does not define.
// The Kuhn meshes of widths h, 2h, 4h, ... are nested.  The prolongation P is
// P1 interpolation: coarse values at coincident nodes, the mean of the two
// end points at the midpoints of coarse edges, which run in the seven
// directions x, y, z, x+y, x+z, y+z, x+y+z.  The Galerkin operator P^T Kx P is
// again the 7-point stencil, with coefficient 2c on the coarse mesh.
//
// The preconditioner is one V-cycle started from zero:
//  - smoothing: two Chebyshev steps on D^{-1} Kx (D = 6c) for [1/3, 2], the
//    part of its spectrum (0, 2) that the coarse mesh cannot represent, before
//    and after the coarse correction;
//  - restriction P^T of the residual (15 fine nodes per coarse node),
//    prolongation P of the correction;
//  - the coarsest level (at most kMG3ExactMax nodes per direction) is solved
//    exactly by the 3-D discrete sine transform: with T = tridiag(-1, 2, -1) =
//    S diag(l) S, Kx = c (T (x) I (x) I + I (x) T (x) I + I (x) I (x) T), so the
//    nodal array U of Kx U = B is S3 [(S3 B) / (c (l_i + l_j + l_k))] with S3
//    the transform along all three axes.  Three launches: a 2-D transform of
//    every z-plane (two 64 x 64 GEMMs on the matrix cores), then per y-plane
//    the transform along z, the division and the inverse transform along z,
//    then the inverse 2-D transform of every z-plane.
// In FP64 the V-cycle is a fixed symmetric positive definite operator (the
// post-smoothing polynomial is the adjoint of the pre-smoothing one), so the
// outer iteration is ordinary preconditioned CG.  The FP32-storage variant
// below is symmetric and linear only up to single-precision rounding.
//
// Shifted operator Kx + s Mx (the rational Krylov steps, Sec. 4): every level
// adds s times its own Q1 mass (rediscretised: the Q1 mass is not a Galerkin
// product of the Kuhn-mesh interpolation), the smoother uses the shifted
// diagonal, and the coarsest solve stays exact because tridiag(1, 4, 1) is
// diagonalised by the same sine transform.
//
// Mixed precision (MGPlan::f32): the same launches store every vector of the
// V-cycle in FP32 except the finest right-hand side (the CG residual) and the
// result (the preconditioned residual), which stay FP64; loads widen to FP64
// and all arithmetic is FP64.  The pre-smoothing launch rounds its input b to
// FP32 in the LDS tile while the post-smoothing launches read b in FP64, so
// the variant is linear and symmetric only up to single-precision rounding.
// The rounding perturbs the preconditioner only, so the FP64 CG around it
// reaches the same tolerances.  The finest level moves 64 bytes per node and
// column (96 with FP64 vectors in the same launches, 58 with the FP64
// V-cycle's fused post-smoothing launch).
//
// Launches per smoothed level: "pre" (both pre-smoothing steps from zero,
// which need b on a one-node halo only, on the tile and its halo, then the
// residual; the iterate and the residual are stored), "restrict" (P^T of the
// residual), "post" (iterate + P e_c on a two-node halo, both
// post-smoothing steps, the result; in the FP32-storage V-cycle two launches,
// "post1" and "post2", one per step).  Fine-level launches work on 32 x 8 x 4
// tiles staged in LDS with a one- or two-node halo.
#include <hip/hip_runtime.h>

#include <cmath>

#include "mg_common.h"
#include "sts_internal.h"

namespace sts {

namespace {

using namespace mgc;

constexpr int kT = 256;
// The pre- and post-smoothing launches run 512 threads on the 32 x 8 x 4
// tile: their FP64 LDS tiles allow five (pre) or four (post) work-groups per
// CU, and with 256 threads that was 20 or 16 waves to hide the serial fill,
// smoothing and store phases of each work-group (measured on the 255^3 grid:
// pre 223 -> 211 ms, post 386 -> 367 ms per solve).
constexpr int kPreT = 512;                             // threads of the pre-smoothing launch
constexpr int kPostT = 512;                            // threads of the fused post-smoothing launch
constexpr int TX = 32, TY = 8, TZ = 4;                 // fine tile
constexpr int RX = TX + 2, RY = TY + 2, RZ = TZ + 2;   // with a one-node halo
constexpr int NR = RX * RY * RZ;
constexpr int CX = 16, CY = 4, CZ = 4;                 // coarse tile of the restriction
constexpr int kCT = 1024;                              // threads of the coarse launches
constexpr int kE = 64;                                 // padded order of the exact solve
constexpr int kEL = kE + 1;                            // LDS row stride
constexpr double kSmoothLo = 1.0 / 3.0;
static_assert(kMG3ExactMax < kE, "exact level fits the padded transform");

struct Tile3 {
  int x0, y0, z0;
};

__device__ __forceinline__ Tile3 tile_of(int t, int ntx, int nty, int sx, int sy, int sz) {
  return Tile3{(t % ntx) * sx, ((t / ntx) % nty) * sy, (t / (ntx * nty)) * sz};
}

// The level operator at LDS point q of an array with rows of X and planes of
// X * Y: c (6 u - sum of the six neighbours), plus with SH the shifted mass
// term sm (1, 4, 1) x (1, 4, 1) x (1, 4, 1) (s Mx, Mx the Q1 mass with
// sm = s (h/6)^3 of the level; the coarse levels rediscretise it).
template <bool SH, int X, int Y, class T>
__device__ __forceinline__ double k7(const T* s, int q, double c, double sm) {
  auto at = [&](int o) { return (double)s[o]; };
  double v = c * (6.0 * at(q) - (at(q - 1) + at(q + 1)) - (at(q - X) + at(q + X)) -
                  (at(q - X * Y) + at(q + X * Y)));
  if (SH) {
    double m = 0.0;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        const int o = q + dz * X * Y + dy * X;
        const double w = (dz == 0 ? 4.0 : 1.0) * (dy == 0 ? 4.0 : 1.0);
        m += w * ((at(o - 1) + at(o + 1)) + 4.0 * at(o));
      }
    }
    v += sm * m;
  }
  return v;
}

// Diagonal of the level operator.
template <bool SH>
__device__ __forceinline__ double k7_diag(double c, double sm) {
  return SH ? 6.0 * c + 64.0 * sm : 6.0 * c;
}

template <int N, class S>
using Staged = StagedN<N, S, kT>;

// Slot i of the tile of g (n^3 nodes, x fastest) with a one-node halo; zero
// outside the domain (the Dirichlet values).
template <class S>
__device__ __forceinline__ S halo_at(const S* g, int n, const Tile3& T, int i) {
  const int gx = T.x0 - 1 + i % RX, gy = T.y0 - 1 + (i / RX) % RY, gz = T.z0 - 1 + i / (RX * RY);
  const bool in = gx >= 0 && gx < n && gy >= 0 && gy < n && gz >= 0 && gz < n;
  return ld_or_zero(g, in, ((size_t)gz * n + gy) * n + gx);
}

template <class S>
__device__ __forceinline__ void load_halo(const S* g, int n, const Tile3& T, S* s) {
  Staged<NR, S> h;
  h.load([&](int i) { return halo_at(g, n, T, i); });
  h.store(s);
}

// The tile nodes of a thread (tile node threadIdx.x + k kT): global index g
// (0 outside the domain, so that loads at g stay branch-free), LDS index q in
// the one-node-halo array, and whether the node is inside.
constexpr int NC = TX * TY * TZ / kT;
static_assert(NC * kT == TX * TY * TZ, "whole tile nodes per thread");
struct Core {
  size_t g[NC];
  int q[NC];
  bool in[NC];
};

__device__ __forceinline__ Core core_nodes(int n, const Tile3& T) {
  Core c;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int i = threadIdx.x + k * kT;
    const int lx = i % TX, ly = (i / TX) % TY, lz = i / (TX * TY);
    const int gx = T.x0 + lx, gy = T.y0 + ly, gz = T.z0 + lz;
    c.in[k] = gx < n && gy < n && gz < n;
    c.g[k] = c.in[k] ? ((size_t)gz * n + gy) * n + gx : 0;
    c.q[k] = ((lz + 1) * RY + ly + 1) * RX + lx + 1;
  }
  return c;
}

// Visit the tile's own nodes: f(global index, LDS index in the halo array).
template <class F>
__device__ __forceinline__ void for_core(int n, const Tile3& T, F&& f) {
  for (int i = threadIdx.x; i < TX * TY * TZ; i += kT) {
    const int lx = i % TX, ly = (i / TX) % TY, lz = i / (TX * TY);
    const int gx = T.x0 + lx, gy = T.y0 + ly, gz = T.z0 + lz;
    if (gx < n && gy < n && gz < n)
      f(((size_t)gz * n + gy) * n + gx, ((lz + 1) * RY + ly + 1) * RX + lx + 1);
  }
}

// Vector types: the fine right-hand side bf and result ef are B, every other
// vector (and both vectors of the coarser levels) S; double / double, or in
// the mixed-precision V-cycle double / float on the finest level and
// float / float below it.  Arithmetic is FP64 throughout.
struct Level3Args {
  int nf, nc;           // fine / coarse nodes per direction (nf = 2 nc + 1)
  int64_t ldf, ldc;     // column strides, in elements
  const void* bf;       // fine right-hand side (B)
  void* xp;             // pre-smoothed iterate: written by pre, read by post (S)
  void* bc;             // restrict: coarse right-hand side (S)
  const void* ec;       // post, post1: coarse correction (S)
  void* u1;             // post1 -> post2: iterate after the first step (S)
  void* d0;             // pre -> restrict: the residual; post1 -> post2: first Chebyshev direction (S)
  void* ef;             // post, post2: result on the fine level (B)
  int ntx, nty, ntz;    // tiles of the launch
  int nlaunch;
  int cols[kMaxCols];
  const CGScal* st;     // per-column activity, may be null (all active)
  double c;             // stencil coefficient of the fine level
  double sm;            // shifted mass scale s (h/6)^3 of the fine level (0: Kx alone)
  double a1, c0, c1;    // Chebyshev coefficients of steps 0 and 1
  double* part;         // post, post2: per-tile (b, e), may be null
  int max_tiles;
};

#define STS_MG3_PROLOGUE(A)                                                    \
  const int ntiles = (A).ntx * (A).nty * (A).ntz;                              \
  const int lin = xcd_remap(blockIdx.x, (A).nlaunch * ntiles);                 \
  const int t = lin / (A).nlaunch, col = (A).cols[lin % (A).nlaunch];          \
  if ((A).st && !(A).st[col].active) return;

// pre: u_1 = c_0 b / D, d_1 = a_1 u_1 + c_1 (b - K u_1) / D, u_2 = u_1 + d_1
// on the tile and a one-node halo (from b on a two-node halo), then the
// residual r = b - K u_2 on the tile.  Stores u_2 (for post) and r.  One LDS
// array holds b first and u_2 after it (the values pass through registers),
// so the launch needs one b tile of LDS (27 KB in FP64).  LDS arrays hold
// the storage type S (b rounded to it in the mixed-precision V-cycle); every
// value is widened to FP64 before it is used.
template <bool SH, class B, class S, int NT>
__global__ __launch_bounds__(NT) void mg3_pre_kernel(Level3Args a) {
  constexpr int BX = TX + 4, BY = TY + 4, BZ = TZ + 4;   // b with a two-node halo
  constexpr int NU = (NR + NT - 1) / NT;                 // halo-1 nodes per thread
  constexpr int NK = TX * TY * TZ / NT;                  // tile nodes per thread
  static_assert(NK * NT == TX * TY * TZ, "whole tile nodes per thread");
  static_assert(NR <= BX * BY * BZ, "u_2 fits where b was");
  __shared__ S sh[BX * BY * BZ];
  STS_MG3_PROLOGUE(a)
  const Tile3 T = tile_of(t, a.ntx, a.nty, TX, TY, TZ);
  const int nf = a.nf;
  const B* bf = static_cast<const B*>(a.bf) + (size_t)col * a.ldf;
  {
    StagedN<BX * BY * BZ, S, NT> hb;
    hb.load([&](int i) {
      const int gx = T.x0 - 2 + i % BX, gy = T.y0 - 2 + (i / BX) % BY, gz = T.z0 - 2 + i / (BX * BY);
      const bool in = gx >= 0 && gx < nf && gy >= 0 && gy < nf && gz >= 0 && gz < nf;
      return (S)ld_or_zero(bf, in, ((size_t)gz * nf + gy) * nf + gx);
    });
    hb.store(sh);
  }
  __syncthreads();
  const double inv_d = 1.0 / k7_diag<SH>(a.c, a.sm);
  double u2r[NU];
#pragma unroll
  for (int k = 0; k < NU; ++k) {
    const int i = threadIdx.x + k * NT;
    double u2 = 0.0;   // zero outside the domain (the Dirichlet values)
    if (i < NR) {
      const int lx = i % RX, ly = (i / RX) % RY, lz = i / (RX * RY);
      const int gx = T.x0 - 1 + lx, gy = T.y0 - 1 + ly, gz = T.z0 - 1 + lz;
      if (gx >= 0 && gx < nf && gy >= 0 && gy < nf && gz >= 0 && gz < nf) {
        const int q = ((lz + 1) * BY + ly + 1) * BX + lx + 1;
        const double b = sh[q];
        const double u1 = a.c0 * inv_d * b;
        const double ku1 = a.c0 * inv_d * k7<SH, BX, BY>(sh, q, a.c, a.sm);
        u2 = u1 + (a.a1 * u1 + a.c1 * inv_d * (b - ku1));
      }
    }
    u2r[k] = u2;
  }
  double bc[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int i = threadIdx.x + k * NT;
    const int lx = i % TX, ly = (i / TX) % TY, lz = i / (TX * TY);
    bc[k] = sh[((lz + 2) * BY + ly + 2) * BX + lx + 2];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NU; ++k) {
    const int i = threadIdx.x + k * NT;
    if (i < NR) sh[i] = (S)u2r[k];
  }
  __syncthreads();
  S* xp = static_cast<S*>(a.xp) + (size_t)col * a.ldf;
  S* r = static_cast<S*>(a.d0) + (size_t)col * a.ldf;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int i = threadIdx.x + k * NT;
    const int lx = i % TX, ly = (i / TX) % TY, lz = i / (TX * TY);
    const int gx = T.x0 + lx, gy = T.y0 + ly, gz = T.z0 + lz;
    if (gx < nf && gy < nf && gz < nf) {
      const size_t g = ((size_t)gz * nf + gy) * nf + gx;
      const int q = ((lz + 1) * RY + ly + 1) * RX + lx + 1;
      xp[g] = (S)sh[q];
      r[g] = (S)(bc[k] - k7<SH, RX, RY>(sh, q, a.c, a.sm));
    }
  }
}

// restrict: b_c = P^T r, the coincident fine node plus half of each of its 14
// neighbours along the seven edge directions, from r on the fine nodes
// around the coarse tile.
template <class S>
__global__ __launch_bounds__(kT) void mg3_restrict_kernel(Level3Args a) {
  constexpr int SX = 2 * CX + 1, SY = 2 * CY + 1, SZ = 2 * CZ + 1;
  __shared__ S rs[SX * SY * SZ];
  STS_MG3_PROLOGUE(a)
  const Tile3 C = tile_of(t, a.ntx, a.nty, CX, CY, CZ);
  const int nf = a.nf, nc = a.nc;
  const int fx0 = 2 * C.x0, fy0 = 2 * C.y0, fz0 = 2 * C.z0;
  const S* r = static_cast<const S*>(a.d0) + (size_t)col * a.ldf;
  {
    Staged<SX * SY * SZ, S> hr;
    hr.load([&](int i) {
      const int gx = fx0 + i % SX, gy = fy0 + (i / SX) % SY, gz = fz0 + i / (SX * SY);
      // fine nodes beyond the domain are never gathered (every coarse node's
      // neighbours lie inside); read them as zero
      return ld_or_zero(r, gx < nf && gy < nf && gz < nf, ((size_t)gz * nf + gy) * nf + gx);
    });
    hr.store(rs);
  }
  __syncthreads();
  S* bc = static_cast<S*>(a.bc) + (size_t)col * a.ldc;
  for (int i = threadIdx.x; i < CX * CY * CZ; i += kT) {
    const int I = C.x0 + i % CX, J = C.y0 + (i / CX) % CY, K = C.z0 + i / (CX * CY);
    if (I < nc && J < nc && K < nc) {
      const int q = ((2 * (K - C.z0) + 1) * SY + 2 * (J - C.y0) + 1) * SX + 2 * (I - C.x0) + 1;
      double s = 0.0;
#pragma unroll
      for (int e = 1; e < 8; ++e) {
        const int o = (e & 1) + ((e >> 1) & 1) * SX + ((e >> 2) & 1) * SX * SY;
        s += (double)rs[q + o] + (double)rs[q - o];
      }
      bc[((size_t)K * nc + J) * nc + I] = (S)((double)rs[q] + 0.5 * s);
    }
  }
}

// P1 interpolation at fine node (gx, gy, gz) from an LDS block of coarse
// values with origin (ox, oy, oz) and dimensions EX x EY.  Per axis, fine
// index 2I+1 coincides with coarse I and an even fine index 2I+2 lies between
// coarse I and I+1; a node even along the axes in a set E is the midpoint of
// the coarse edge from (I, J, K) in direction E.
template <int EX, int EY, class S>
__device__ __forceinline__ double interp3(const S* es, int ox, int oy, int oz, int gx, int gy,
                                          int gz) {
  const int ex = (gx & 1) ^ 1, ey = (gy & 1) ^ 1, ez = (gz & 1) ^ 1;
  const int I = (gx - 1 - ex) >> 1, J = (gy - 1 - ey) >> 1, K = (gz - 1 - ez) >> 1;
  const S* c = es + ((K - oz) * EY + (J - oy)) * EX + (I - ox);
  if ((ex | ey | ez) == 0) return (double)c[0];
  return 0.5 * ((double)c[0] + (double)c[ex + ey * EX + ez * EX * EY]);
}

// post: u = u_2 + P e_c on the tile and a two-node halo; the first step
// d_0 = c_0 (b - K u) / D, u_1 = u + d_0 on the tile and a one-node halo;
// the second step d_1 = a_1 d_0 + c_1 (b - K u_1) / D, e = u_1 + d_1 on the
// tile; per-tile (b, e).  Every work-group computes the first step on its
// halo itself (the same arithmetic its neighbour does for those nodes), so
// u_1 and d_0 never go through global memory.  One LDS array holds u first,
// then u_1 on the one-node halo followed by d_0 on the tile (the values pass
// through registers).  u_1 and d_0 are rounded to the storage type S, as
// stored vectors would be.
template <bool SH, class B, class S, int NT>
__global__ __launch_bounds__(NT) void mg3_post_kernel(Level3Args a) {
  constexpr int BX = TX + 4, BY = TY + 4, BZ = TZ + 4;   // u with a two-node halo
  constexpr int EX = TX / 2 + 3, EY = TY / 2 + 3, EZ = TZ / 2 + 3;
  constexpr int NU = (NR + NT - 1) / NT;                 // halo-1 nodes per thread
  constexpr int NK = TX * TY * TZ / NT;                  // tile nodes per thread
  static_assert(NK * NT == TX * TY * TZ, "whole tile nodes per thread");
  static_assert(NR + TX * TY * TZ <= BX * BY * BZ, "u_1 and d_0 fit where u was");
  __shared__ S sh[BX * BY * BZ];
  __shared__ S es[EX * EY * EZ];
  __shared__ double red[NT / 64];
  STS_MG3_PROLOGUE(a)
  const Tile3 T = tile_of(t, a.ntx, a.nty, TX, TY, TZ);
  const int nf = a.nf, nc = a.nc;
  // coarse nodes under the two-node halo: fine x0 - 2 interpolates from
  // coarse x0 / 2 - 2, fine x0 + TX + 1 from coarse x0 / 2 + TX / 2
  const int ox = T.x0 / 2 - 2, oy = T.y0 / 2 - 2, oz = T.z0 / 2 - 2;
  const S* xp = static_cast<const S*>(a.xp) + (size_t)col * a.ldf;
  const S* ec = static_cast<const S*>(a.ec) + (size_t)col * a.ldc;
  const B* bf = static_cast<const B*>(a.bf) + (size_t)col * a.ldf;
  auto inside = [&](int gx, int gy, int gz) {
    return gx >= 0 && gx < nf && gy >= 0 && gy < nf && gz >= 0 && gz < nf;
  };
  // every global read of the launch in flight before the first wait:
  // u_2 on the two-node halo, e_c, b on the one-node halo and on the tile
  StagedN<BX * BY * BZ, S, NT> hx;
  StagedN<EX * EY * EZ, S, NT> he;
  hx.load([&](int i) {
    const int gx = T.x0 - 2 + i % BX, gy = T.y0 - 2 + (i / BX) % BY, gz = T.z0 - 2 + i / (BX * BY);
    return ld_or_zero(xp, inside(gx, gy, gz), ((size_t)gz * nf + gy) * nf + gx);
  });
  he.load([&](int i) {
    const int I = ox + i % EX, J = oy + (i / EX) % EY, K = oz + i / (EX * EY);
    const bool in = I >= 0 && I < nc && J >= 0 && J < nc && K >= 0 && K < nc;
    return ld_or_zero(ec, in, ((size_t)K * nc + J) * nc + I);
  });
  StagedN<NR, B, NT> hb;
  hb.load([&](int i) { return halo_at(bf, nf, T, i); });
  size_t cg[NK];
  int cq[NK];
  bool cin[NK];
  B bv[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int i = threadIdx.x + k * NT;
    const int lx = i % TX, ly = (i / TX) % TY, lz = i / (TX * TY);
    const int gx = T.x0 + lx, gy = T.y0 + ly, gz = T.z0 + lz;
    cin[k] = gx < nf && gy < nf && gz < nf;
    cg[k] = cin[k] ? ((size_t)gz * nf + gy) * nf + gx : 0;
    cq[k] = ((lz + 1) * RY + ly + 1) * RX + lx + 1;
    bv[k] = bf[cg[k]];
  }
  hx.store(sh);
  he.store(es);
  __syncthreads();
  // u = u_2 + P e_c (each thread updates its own slots)
#pragma unroll
  for (int k = 0; k < StagedN<BX * BY * BZ, S, NT>::NI; ++k) {
    const int i = threadIdx.x + k * NT;
    if (i < BX * BY * BZ) {
      const int gx = T.x0 - 2 + i % BX, gy = T.y0 - 2 + (i / BX) % BY, gz = T.z0 - 2 + i / (BX * BY);
      if (inside(gx, gy, gz))
        sh[i] = (S)((double)sh[i] + interp3<EX, EY>(es, ox, oy, oz, gx, gy, gz));
    }
  }
  __syncthreads();
  // first step on the tile and its one-node halo (zero outside the domain)
  const double inv_d = 1.0 / k7_diag<SH>(a.c, a.sm);
  S u1r[NU], d0r[NU];
#pragma unroll
  for (int k = 0; k < NU; ++k) {
    const int i = threadIdx.x + k * NT;
    S u1 = (S)0, d0 = (S)0;
    if (i < NR) {
      const int lx = i % RX, ly = (i / RX) % RY, lz = i / (RX * RY);
      if (inside(T.x0 - 1 + lx, T.y0 - 1 + ly, T.z0 - 1 + lz)) {
        const int q = ((lz + 1) * BY + ly + 1) * BX + lx + 1;
        const double d = a.c0 * inv_d * ((double)hb.v[k] - k7<SH, BX, BY>(sh, q, a.c, a.sm));
        d0 = (S)d;
        u1 = (S)((double)sh[q] + d);
      }
    }
    u1r[k] = u1;
    d0r[k] = d0;
  }
  __syncthreads();
  S* d0s = sh + NR;   // d_0 on the tile, x fastest
#pragma unroll
  for (int k = 0; k < NU; ++k) {
    const int i = threadIdx.x + k * NT;
    if (i < NR) {
      sh[i] = u1r[k];
      const int lx = i % RX - 1, ly = (i / RX) % RY - 1, lz = i / (RX * RY) - 1;
      if (lx >= 0 && lx < TX && ly >= 0 && ly < TY && lz >= 0 && lz < TZ)
        d0s[(lz * TY + ly) * TX + lx] = d0r[k];
    }
  }
  __syncthreads();
  // second step on the tile
  B* ef = static_cast<B*>(a.ef) + (size_t)col * a.ldf;
  double part = 0.0;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    if (!cin[k]) continue;
    const int q = cq[k];
    const double b = bv[k];
    const double d0 = d0s[threadIdx.x + k * NT];
    const double e =
        (double)sh[q] + (a.a1 * d0 + a.c1 * inv_d * (b - k7<SH, RX, RY>(sh, q, a.c, a.sm)));
    ef[cg[k]] = (B)e;
    part += b * (double)(B)e;   // (b, e) of the stored result
  }
  if (a.part) {
    part = block_sum<NT>(part, red);
    if (threadIdx.x == 0) a.part[(size_t)col * a.max_tiles + t] = part;
  }
}

// The same two post-smoothing steps as two launches, for the FP32-storage
// V-cycle: there the recomputation on the halo that the fused launch does
// costs more than the stored u_1 and d_0 it saves (all arithmetic is FP64
// while the vectors move half the bytes).
// post1: u = u_2 + P e_c on the tile and its halo; d_0 = c_0 (b - K u) / D,
// u_1 = u + d_0 on the tile.
template <bool SH, class B, class S>
__global__ __launch_bounds__(kT) void mg3_post1_kernel(Level3Args a) {
  constexpr int EX = TX / 2 + 2, EY = TY / 2 + 2, EZ = TZ / 2 + 2;
  __shared__ S us[NR];
  __shared__ S es[EX * EY * EZ];
  STS_MG3_PROLOGUE(a)
  const Tile3 T = tile_of(t, a.ntx, a.nty, TX, TY, TZ);
  const int nf = a.nf, nc = a.nc;
  const int ox = T.x0 / 2 - 1, oy = T.y0 / 2 - 1, oz = T.z0 / 2 - 1;
  const S* xp = static_cast<const S*>(a.xp) + (size_t)col * a.ldf;
  const S* ec = static_cast<const S*>(a.ec) + (size_t)col * a.ldc;
  const B* bf = static_cast<const B*>(a.bf) + (size_t)col * a.ldf;
  // every global read of the launch in flight before the first wait
  Staged<NR, S> hu;
  Staged<EX * EY * EZ, S> he;
  hu.load([&](int i) { return halo_at(xp, nf, T, i); });
  he.load([&](int i) {
    const int I = ox + i % EX, J = oy + (i / EX) % EY, K = oz + i / (EX * EY);
    const bool in = I >= 0 && I < nc && J >= 0 && J < nc && K >= 0 && K < nc;
    return ld_or_zero(ec, in, ((size_t)K * nc + J) * nc + I);
  });
  const Core C = core_nodes(nf, T);
  B bv[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) bv[k] = bf[C.g[k]];
  hu.store(us);
  he.store(es);
  __syncthreads();
  for (int i = threadIdx.x; i < NR; i += kT) {
    const int gx = T.x0 - 1 + i % RX, gy = T.y0 - 1 + (i / RX) % RY, gz = T.z0 - 1 + i / (RX * RY);
    if (gx >= 0 && gx < nf && gy >= 0 && gy < nf && gz >= 0 && gz < nf)
      us[i] = (S)((double)us[i] + interp3<EX, EY>(es, ox, oy, oz, gx, gy, gz));
  }
  __syncthreads();
  const double inv_d = 1.0 / k7_diag<SH>(a.c, a.sm);
  S* u1 = static_cast<S*>(a.u1) + (size_t)col * a.ldf;
  S* d0 = static_cast<S*>(a.d0) + (size_t)col * a.ldf;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    if (!C.in[k]) continue;
    const int q = C.q[k];
    const double d = a.c0 * inv_d * ((double)bv[k] - k7<SH, RX, RY>(us, q, a.c, a.sm));
    d0[C.g[k]] = (S)d;
    u1[C.g[k]] = (S)((double)us[q] + d);
  }
}

// post2: d_1 = a_1 d_0 + c_1 (b - K u_1) / D, e = u_1 + d_1; per-tile (b, e).
template <bool SH, class B, class S>
__global__ __launch_bounds__(kT) void mg3_post2_kernel(Level3Args a) {
  __shared__ S us[NR];
  __shared__ double red[kT / 64];
  STS_MG3_PROLOGUE(a)
  const Tile3 T = tile_of(t, a.ntx, a.nty, TX, TY, TZ);
  const int nf = a.nf;
  const S* u1 = static_cast<const S*>(a.u1) + (size_t)col * a.ldf;
  const B* bf = static_cast<const B*>(a.bf) + (size_t)col * a.ldf;
  const S* d0 = static_cast<const S*>(a.d0) + (size_t)col * a.ldf;
  // every global read of the launch in flight before the first wait
  Staged<NR, S> hu;
  hu.load([&](int i) { return halo_at(u1, nf, T, i); });
  const Core C = core_nodes(nf, T);
  B bv[NC];
  S dv[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    bv[k] = bf[C.g[k]];
    dv[k] = d0[C.g[k]];
  }
  hu.store(us);
  __syncthreads();
  const double inv_d = 1.0 / k7_diag<SH>(a.c, a.sm);
  B* ef = static_cast<B*>(a.ef) + (size_t)col * a.ldf;
  double part = 0.0;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    if (!C.in[k]) continue;
    const int q = C.q[k];
    const double b = bv[k];
    const double e =
        (double)us[q] + (a.a1 * (double)dv[k] + a.c1 * inv_d * (b - k7<SH, RX, RY>(us, q, a.c, a.sm)));
    ef[C.g[k]] = (B)e;
    part += b * (double)(B)e;   // (b, e) of the stored result
  }
  if (a.part) {
    part = block_sum<kT>(part, red);
    if (threadIdx.x == 0) a.part[(size_t)col * a.max_tiles + t] = part;
  }
}

// ---------------------------------------------------------------------------
// exact coarse solve by the 3-D sine transform (order m <= kMG3ExactMax)
// ---------------------------------------------------------------------------
// in / out / rhs hold T (double, or float in the mixed-precision V-cycle).
struct Coarse3Args {
  int m;
  int64_t ld;
  const void* in;       // per column, m^3 (x fastest)
  void* out;
  const void* rhs;      // last stage with partials: the right-hand side b
  const double* dst;    // S (m x m, symmetric), then l (m)
  double c;             // stencil coefficient of the coarse level
  double sm;            // shifted mass scale of the coarse level (0: Kx alone)
  int nlaunch;
  int cols[kMaxCols];
  const CGScal* st;
  double* part;         // (b, e) per plane when the exact solve is the whole V-cycle
  int max_tiles;
};

// C = A B for 64 x 64 LDS matrices (row stride kEL), one 16 x 16 tile per
// wave; `epi(y, x, v)` gives the stored value.
template <class Epi>
__device__ __forceinline__ void lds_gemm64(const double* A, const double* B, double* C, Epi&& epi) {
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
    C[y * kEL + x] = epi(y, x, sum[q]);
  }
}

// Stage 0 / 2: every z-plane P (y rows, x columns) becomes S P S.
template <class T>
__global__ __launch_bounds__(kCT) void coarse3_plane_kernel(Coarse3Args a) {
  __shared__ double S[kE * kEL];
  __shared__ double X[kE * kEL];
  __shared__ double Tm[kE * kEL];
  __shared__ double red[kCT / 64];
  const int col = a.cols[blockIdx.y];
  if (a.st && !a.st[col].active) return;
  const int m = a.m, z = blockIdx.x;
  const size_t off = (size_t)col * a.ld + (size_t)z * m * m;
  const T* in = static_cast<const T*>(a.in) + off;
  for (int i = threadIdx.x; i < kE * kE; i += kCT) {
    const int y = i / kE, x = i % kE;
    const bool ok = y < m && x < m;
    S[y * kEL + x] = ok ? a.dst[y * m + x] : 0.0;
    X[y * kEL + x] = ok ? (double)in[y * m + x] : 0.0;
  }
  __syncthreads();
  auto keep = [](int, int, double v) { return v; };
  lds_gemm64(S, X, Tm, keep);
  __syncthreads();
  lds_gemm64(Tm, S, X, keep);
  __syncthreads();
  T* out = static_cast<T*>(a.out) + off;
  double part = 0.0;
  for (int i = threadIdx.x; i < m * m; i += kCT) {
    const double v = X[(i / m) * kEL + i % m];
    out[i] = (T)v;
    if (a.part) part += (double)static_cast<const T*>(a.rhs)[off + i] * v;
  }
  if (a.part) {
    part = block_sum<kCT>(part, red);
    if (threadIdx.x == 0) a.part[(size_t)col * a.max_tiles + z] = part;
  }
}

// Stage 1: every y-plane Q (z rows, x columns) becomes
// S [(S Q) / (c (l_z + l_y + l_x))], in place.
template <class T>
__global__ __launch_bounds__(kCT) void coarse3_z_kernel(Coarse3Args a) {
  __shared__ double S[kE * kEL];
  __shared__ double X[kE * kEL];
  __shared__ double Tm[kE * kEL];
  __shared__ double l[kE];
  const int col = a.cols[blockIdx.y];
  if (a.st && !a.st[col].active) return;
  const int m = a.m, y = blockIdx.x;
  T* io = static_cast<T*>(a.out) + (size_t)col * a.ld;
  for (int i = threadIdx.x; i < kE * kE; i += kCT) {
    const int r = i / kE, x = i % kE;
    const bool ok = r < m && x < m;
    S[r * kEL + x] = ok ? a.dst[r * m + x] : 0.0;
    X[r * kEL + x] = ok ? (double)io[((size_t)r * m + y) * m + x] : 0.0;
  }
  if (threadIdx.x < kE) l[threadIdx.x] = threadIdx.x < m ? a.dst[(size_t)m * m + threadIdx.x] : 0.0;
  __syncthreads();
  // Kx + s Mx in the sine basis: c (l_z + l_y + l_x) + sm (6 - l_z)(6 - l_y)(6 - l_x)
  // (tridiag(1, 4, 1) = 6 I - tridiag(-1, 2, -1))
  const double ly = l[y], c = a.c, sm = a.sm;
  lds_gemm64(S, X, Tm, [&](int r, int x, double v) {
    return (r < m && x < m)
               ? v / (c * (l[r] + ly + l[x]) + sm * ((6.0 - l[r]) * (6.0 - ly) * (6.0 - l[x])))
               : 0.0;
  });
  __syncthreads();
  lds_gemm64(S, Tm, X, [](int, int, double v) { return v; });
  __syncthreads();
  for (int i = threadIdx.x; i < m * m; i += kCT) {
    const int r = i / m, x = i % m;
    io[((size_t)r * m + y) * m + x] = (T)X[r * kEL + x];
  }
}

// ---------------------------------------------------------------------------
// PCG launches on the finest grid (tiles TX x TY x TZ)
// ---------------------------------------------------------------------------
// The vectors x, r, z, p and q hold V: double, or float in the FP32 PCG of
// the mixed-precision inner solves, where the vector arithmetic (the stencil
// product q = K p, the updates and the per-tile inner products) runs in FP32
// too.  The CG scalars (alpha, beta, rho) and the cross-tile sums of the
// per-tile partials stay FP64.
struct PCG3Args {
  int n;
  int64_t ld;
  int ntx, nty, ntz;
  int ncols;
  int nlaunch;
  int cols[kMaxCols];
  double c;
  double sm;
  void* x;
  int64_t ldx;
  void* r;
  const void* z;
  const void* pin;
  void* pout;
  void* q;
  const CGScal* prev;
  CGScal* next;
  double* part_rr;
  double* part_rz;
  double* part_pq;
  int rz_tiles;
  double* alpha;
  int max_tiles;
  const double* tot;   // (r, r), (r, z), (p, q) per column (3 x kMaxCols), or null:
                       // each work-group then adds the per-tile partials itself
  const double* b[kMaxCols];
  double rtol2[kMaxCols];   // set-up: squared relative tolerance per column
};

// Large grids: one work-group per column and quantity adds the per-tile
// partials (fixed order) so that the PCG launches read one total each.
constexpr int kSplitReduceTiles = 1024;

struct Reduce3Args {
  const double* part[2];   // partial arrays, column stride max_tiles
  int count[2];            // partials per column
  double* out[2];          // totals per column
  int max_tiles;
  int cols[kMaxCols];
};

__global__ __launch_bounds__(kT) void pcg3_reduce_kernel(Reduce3Args a) {
  __shared__ double red[kT / 64];
  const int col = a.cols[blockIdx.x], q = blockIdx.y;
  const double* p = a.part[q] + (size_t)col * a.max_tiles;
  double s = 0.0;
  // unrolled so that eight loads are in flight per trip (same summation order)
#pragma unroll 8
  for (int u = threadIdx.x; u < a.count[q]; u += kT) s += p[u];
  s = block_sum<kT>(s, red);
  if (threadIdx.x == 0) a.out[q][col] = s;
}

// Work-group sum in the vector type (FP32 sums for the FP32 PCG).
__device__ __forceinline__ float wave_sum_v(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_sum_v(double v) { return wave_sum(v); }

template <class V>
__device__ __forceinline__ double block_sum_v(V v, V* red) {
  v = wave_sum_v(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  V s = (V)0;
#pragma unroll
  for (int w = 0; w < kT / 64; ++w) s += red[w];
  __syncthreads();
  return (double)s;
}

// q = K p in the vector type: FP64 as in the V-cycle, or FP32 arithmetic.
template <bool SH, class V>
__device__ __forceinline__ V k7_vec(const V* s, int q, double c, double sm) {
  if constexpr (sizeof(V) == 8) {
    return k7<SH, RX, RY>(s, q, c, sm);
  } else {
    const float cf = (float)c;
    float v = cf * (6.0f * s[q] - (s[q - 1] + s[q + 1]) - (s[q - RX] + s[q + RX]) -
                    (s[q - RX * RY] + s[q + RX * RY]));
    if (SH) {
      float m = 0.0f;
#pragma unroll
      for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
          const int o = q + dz * RX * RY + dy * RX;
          const float w = (dz == 0 ? 4.0f : 1.0f) * (dy == 0 ? 4.0f : 1.0f);
          m += w * ((s[o - 1] + s[o + 1]) + 4.0f * s[o]);
        }
      }
      v += (float)sm * m;
    }
    return v;
  }
}

#define STS_PCG3_PROLOGUE(A)                                                   \
  const int ntiles = (A).ntx * (A).nty * (A).ntz;                              \
  const int lin = xcd_remap(blockIdx.x, (A).nlaunch * ntiles);                 \
  const int t = lin / (A).nlaunch, jb = lin % (A).nlaunch, col = (A).cols[jb]; \
  (void)jb;                                                                    \
  const Tile3 T = tile_of(t, (A).ntx, (A).nty, TX, TY, TZ);

// A: stopping test and beta; p = z + beta p; q = K p; (p, q).
template <bool SH, class V>
__global__ __launch_bounds__(kT) void pcg3_a_kernel(PCG3Args a) {
  __shared__ V ps[NR];
  __shared__ double red[2][kT / 64];
  __shared__ V redv[kT / 64];
  STS_PCG3_PROLOGUE(a)
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
  double rr = 0.0, rz = 0.0;
  if (a.tot) {
    rr = a.tot[col];
    rz = a.tot[kMaxCols + col];
  } else {
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
  }
  double beta;
  const bool go = pcg_decide(s, rr, rz, a.alpha[col], beta);
  if (t == 0 && threadIdx.x == 0) a.next[col] = s;
  if (!go) return;
  const int n = a.n;
  const V* zg = static_cast<const V*>(a.z) + (size_t)col * a.ld;
  const V* pin = static_cast<const V*>(a.pin) + (size_t)col * a.ld;
  const V bv = (V)beta;
  {
    Staged<NR, V> hp;
    hp.load([&](int i) { return halo_at(zg, n, T, i) + bv * halo_at(pin, n, T, i); });
    hp.store(ps);
  }
  __syncthreads();
  V* pout = static_cast<V*>(a.pout) + (size_t)col * a.ld;
  V* qg = static_cast<V*>(a.q) + (size_t)col * a.ld;
  V part = (V)0;
  for_core(n, T, [&](size_t g, int q) {
    const V pv = ps[q];
    const V qv = k7_vec<SH, V>(ps, q, a.c, a.sm);
    pout[g] = pv;
    qg[g] = qv;
    part += pv * qv;
  });
  const double tot = block_sum_v<V>(part, redv);
  if (threadIdx.x == 0) a.part_pq[(size_t)col * a.max_tiles + t] = tot;
}

// B: alpha = rho / (p, q); x += alpha p; r -= alpha q; (r, r).  x holds XT
// (V, or FP64 for the FP32 PCG whose residual is replaced from x).
template <class V, class XT>
__global__ __launch_bounds__(kT) void pcg3_b_kernel(PCG3Args a) {
  __shared__ double red[kT / 64];
  __shared__ V redv[kT / 64];
  STS_PCG3_PROLOGUE(a)
  const CGScal s = a.next[col];
  if (!s.active) return;
  double pq = 0.0;
  if (a.tot) {
    pq = a.tot[2 * kMaxCols + col];
  } else {
    const double* ppq = a.part_pq + (size_t)col * a.max_tiles;
    for (int u = threadIdx.x; u < ntiles; u += kT) pq += ppq[u];
    pq = block_sum<kT>(pq, red);
  }
  const bool ok = pq > 0.0 && __builtin_isfinite(pq);
  const double alpha = ok ? s.rho / pq : 0.0;
  if (t == 0 && threadIdx.x == 0) a.alpha[col] = alpha;
  if (!ok) return;
  XT* xg = static_cast<XT*>(a.x) + (size_t)col * a.ldx;
  V* rg = static_cast<V*>(a.r) + (size_t)col * a.ld;
  const V* pg = static_cast<const V*>(a.pout) + (size_t)col * a.ld;
  const V* qg = static_cast<const V*>(a.q) + (size_t)col * a.ld;
  const V av = (V)alpha;
  const Core C = core_nodes(a.n, T);
  XT xv[NC];
  V pv[NC], rv[NC], qv[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    xv[k] = xg[C.g[k]];
    pv[k] = pg[C.g[k]];
    rv[k] = rg[C.g[k]];
    qv[k] = qg[C.g[k]];
  }
  V part = (V)0;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    if (!C.in[k]) continue;
    xg[C.g[k]] = xv[k] + (XT)alpha * (XT)pv[k];
    const V r = rv[k] - av * qv[k];
    rg[C.g[k]] = r;
    part += r * r;
  }
  const double tot = block_sum_v<V>(part, redv);
  if (threadIdx.x == 0) a.part_rr[(size_t)col * a.max_tiles + t] = tot;
}

// Set-up: x = 0, r = b (rounded to V), both p buffers 0, partials of (r, r);
// both state slots initialised (columns in the launch list active), alpha = 1.
template <class V, class XT>
__global__ __launch_bounds__(kT) void pcg3_setup_kernel(PCG3Args a, int maxit) {
  __shared__ V redv[kT / 64];
  STS_PCG3_PROLOGUE(a)
  const double* bg = a.b[jb];
  XT* xa = static_cast<XT*>(a.x);
  V* ra = static_cast<V*>(a.r);
  V* pa = static_cast<V*>(const_cast<void*>(a.pin));
  V* pb = static_cast<V*>(a.pout);
  V part = (V)0;
  for_core(a.n, T, [&](size_t g, int) {
    const V bv = (V)bg[g];
    xa[g + (size_t)col * a.ldx] = (XT)0;
    ra[g + (size_t)col * a.ld] = bv;
    pa[g + (size_t)col * a.ld] = (V)0;
    pb[g + (size_t)col * a.ld] = (V)0;
    part += bv * bv;
  });
  const double tot = block_sum_v<V>(part, redv);
  if (threadIdx.x == 0) a.part_rr[(size_t)col * a.max_tiles + t] = tot;
  if (blockIdx.x == 0 && threadIdx.x < kMaxCols) {
    const int c = threadIdx.x;
    bool launched = false;
    for (int j = 0; j < a.nlaunch; ++j) launched |= a.cols[j] == c;
    CGScal s{};
    s.rtol2 = a.rtol2[c];
    s.maxit = maxit;
    s.active = launched ? 1 : 0;
    a.next[c] = s;
    const_cast<CGScal*>(a.prev)[c] = s;
    a.alpha[c] = 1.0;
  }
}

// Defect correction of the FP32 inner solves, in FP64: x += d (one
// elementwise launch; the stencil launch after it reads x on halos that other
// work-groups own, so x must not change under it), then r = b - (Kx + s Mx) x
// and the per-tile partials of (r, r), for the columns of the launch slots
// (own pointers per slot: x FP64, d FP32 or FP64, b and r FP64).
struct Defect3Args {
  int n;
  int ntx, nty, ntz;
  int nlaunch;
  double c, sm;
  double* x[kMaxCols];
  const void* d[kMaxCols];   // null: x unchanged
  const double* b[kMaxCols];
  double* r[kMaxCols];
  double* part;              // per-tile (r, r), slot stride max_tiles
  int max_tiles;
};

template <class D>
__global__ __launch_bounds__(kT) void add_corr3_kernel(Defect3Args a, int64_t nn) {
  const int jb = blockIdx.y;
  const D* d = static_cast<const D*>(a.d[jb]);
  if (!d) return;
  double* x = a.x[jb];
  for (int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x; g < nn; g += (int64_t)gridDim.x * kT)
    x[g] += (double)d[g];
}

template <bool SH>
__global__ __launch_bounds__(kT) void defect3_kernel(Defect3Args a) {
  __shared__ double us[NR];
  __shared__ double red[kT / 64];
  const int ntiles = a.ntx * a.nty * a.ntz;
  const int lin = xcd_remap(blockIdx.x, a.nlaunch * ntiles);
  const int t = lin / a.nlaunch, jb = lin % a.nlaunch;
  const Tile3 T = tile_of(t, a.ntx, a.nty, TX, TY, TZ);
  load_halo(a.x[jb], a.n, T, us);
  __syncthreads();
  const double* bg = a.b[jb];
  double* rg = a.r[jb];
  double part = 0.0;
  const Core C = core_nodes(a.n, T);
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    if (!C.in[k]) continue;
    const double rv = bg[C.g[k]] - k7<SH, RX, RY>(us, C.q[k], a.c, a.sm);
    rg[C.g[k]] = rv;
    part += rv * rv;
  }
  part = block_sum<kT>(part, red);
  if (threadIdx.x == 0) a.part[(size_t)jb * a.max_tiles + t] = part;
}

// Residual replacement of the FP32 PCG: r = b - (Kx + s Mx) x from the FP64
// iterate, stored in FP32, (r, r) per tile in FP64.
struct Replace3Args {
  int n;
  int64_t ld, ldx;
  int ntx, nty, ntz;
  int nlaunch;
  int cols[kMaxCols];
  double c, sm;
  const double* x;
  const double* b[kMaxCols];   // by column
  float* r;
  double* part;
  int max_tiles;
};

template <bool SH>
__global__ __launch_bounds__(kT) void replace3_kernel(Replace3Args a) {
  __shared__ double us[NR];
  __shared__ double red[kT / 64];
  const int ntiles = a.ntx * a.nty * a.ntz;
  const int lin = xcd_remap(blockIdx.x, a.nlaunch * ntiles);
  const int t = lin / a.nlaunch, col = a.cols[lin % a.nlaunch];
  const Tile3 T = tile_of(t, a.ntx, a.nty, TX, TY, TZ);
  load_halo(a.x + (size_t)col * a.ldx, a.n, T, us);
  __syncthreads();
  const double* bg = a.b[col];
  float* rg = a.r + (size_t)col * a.ld;
  double part = 0.0;
  const Core C = core_nodes(a.n, T);
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    if (!C.in[k]) continue;
    const double rv = bg[C.g[k]] - k7<SH, RX, RY>(us, C.q[k], a.c, a.sm);
    rg[C.g[k]] = (float)rv;
    part += rv * rv;
  }
  part = block_sum<kT>(part, red);
  if (threadIdx.x == 0) a.part[(size_t)col * a.max_tiles + t] = part;
}

int tiles3(int n, int sx, int sy, int sz) {
  return ((n + sx - 1) / sx) * ((n + sy - 1) / sy) * ((n + sz - 1) / sz);
}

double level_coef(const MGPlan& p, int l) { return std::ldexp(p.mu, l); }

PCG3Args pcg3_args(const MGWork& w, int parity, const int* cols, int nlaunch, int ncols) {
  PCG3Args a{};
  a.n = w.plan.n[0];
  a.ld = w.ld[0];
  a.ntx = (a.n + TX - 1) / TX;
  a.nty = (a.n + TY - 1) / TY;
  a.ntz = (a.n + TZ - 1) / TZ;
  a.ncols = ncols;
  a.nlaunch = nlaunch;
  for (int j = 0; j < nlaunch; ++j) a.cols[j] = cols[j];
  a.c = w.plan.mu;
  a.sm = w.plan.sw0;
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
  a.rz_tiles = w.plan.nlev > 0 ? tiles3(a.n, TX, TY, TZ) : w.plan.n[0];
  a.alpha = w.alpha;
  a.max_tiles = w.max_tiles;
  return a;
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

bool mg3_plan(const Grid& g, const Stencil& K, MGPlan* plan) {
  if (g.dim != 3 || g.nx != g.ny || g.nx != g.nz || g.nx < 1) return false;
  // Kx must be c times the 7-point pattern (6; -1 x 6); the centre 6 c may
  // differ from six times the neighbour coefficient by rounding
  const double c = -K.c[12];
  if (!(c > 0.0) || std::fabs(K.c[13] - 6.0 * c) > 1e-15 * 6.0 * c) return false;
  for (int i = 0; i < 27; ++i) {
    if (i == 13) continue;
    const double want = (i == 12 || i == 14 || i == 10 || i == 16 || i == 4 || i == 22) ? -c : 0.0;
    if (K.c[i] != want) return false;
  }
  MGPlan p{};
  p.dim = 3;
  p.mu = c;
  int L = 0, n = g.nx;
  p.n[0] = n;
  while (n > kMG3ExactMax) {
    if ((n & 1) == 0 || L + 1 >= kMGMaxLevels) return false;   // does not halve
    n = (n - 1) / 2;
    p.n[++L] = n;
  }
  p.nlev = L;
  p.exact = n;
  *plan = p;
  return true;
}

int mg3_max_tiles(const MGPlan& p) {
  int t = tiles3(p.n[0], TX, TY, TZ);
  if (p.nlev == 0) t = std::max(t, p.n[0]);
  return std::max(t, 1);
}

double mg3_bytes_per_node(const MGPlan& p) {
  const double n0 = std::pow((double)p.n[0], 3);
  const bool all32 = p.f32cg && p.nlev > 0, f32 = (p.f32 || p.f32cg) && p.nlev > 0;
  double b = (all32 ? (p.x64 ? 48.0 : 40.0) : 80.0) * n0;   // PCG A and B
  for (int l = 0; l < p.nlev; ++l) {
    const double nf = std::pow((double)p.n[l], 3), nc = std::pow((double)p.n[l + 1], 3);
    const double sb = (f32 && (l > 0 || all32)) ? 4.0 : 8.0, ss = f32 ? 4.0 : 8.0;
    // pre: b -> xp, r; restrict: r -> b_c; then with FP64 vectors post: xp,
    // b, e_c -> e, with FP32 ones post1: xp, b, e_c -> d0, u1 and post2: u1,
    // b, d0 -> e
    b += (sb + 2.0 * ss) * nf + ss * (nf + nc);
    b += f32 ? ((sb + 3.0 * ss) * nf + ss * nc) + (2.0 * sb + 2.0 * ss) * nf
             : (2.0 * sb + ss) * nf + ss * nc;
  }
  b += (f32 ? 24.0 : 48.0) * std::pow((double)p.exact, 3);
  return b / n0;
}

namespace {

// The smoothed levels' launches with fine vectors B and the others S.
template <class B, class S>
void level_down(Level3Args a, bool shifted, int nlaunch, hipStream_t st) {
  const double nf = std::pow((double)a.nf, 3), nc = std::pow((double)a.nc, 3);
  const double sb = sizeof(B), ss = sizeof(S);
  a.ntx = (a.nf + TX - 1) / TX;
  a.nty = (a.nf + TY - 1) / TY;
  a.ntz = (a.nf + TZ - 1) / TZ;
  int blocks = a.ntx * a.nty * a.ntz * nlaunch;
  const double pre = (sb + 2.0 * ss) * nf * nlaunch;
  if (shifted)
    launch(STS_K_MG_DOWN, pre, mg3_pre_kernel<true, B, S, kPreT>, dim3(blocks), dim3(kPreT), 0, st,
           a);
  else
    launch(STS_K_MG_DOWN, pre, mg3_pre_kernel<false, B, S, kPreT>, dim3(blocks), dim3(kPreT), 0, st,
           a);
  STS_HIP(hipGetLastError());
  a.ntx = (a.nc + CX - 1) / CX;
  a.nty = (a.nc + CY - 1) / CY;
  a.ntz = (a.nc + CZ - 1) / CZ;
  blocks = a.ntx * a.nty * a.ntz * nlaunch;
  launch(STS_K_MG_RESTRICT, ss * (nf + nc) * nlaunch, mg3_restrict_kernel<S>, dim3(blocks),
         dim3(kT), 0, st, a);
  STS_HIP(hipGetLastError());
}

template <class B, class S>
void level_up(Level3Args a, bool shifted, int nlaunch, hipStream_t st) {
  const double nf = std::pow((double)a.nf, 3), nc = std::pow((double)a.nc, 3);
  const double sb = sizeof(B), ss = sizeof(S);
  a.ntx = (a.nf + TX - 1) / TX;
  a.nty = (a.nf + TY - 1) / TY;
  a.ntz = (a.nf + TZ - 1) / TZ;
  const int blocks = a.ntx * a.nty * a.ntz * nlaunch;
  if constexpr (sizeof(S) == 8) {
    const double post = ((2.0 * sb + ss) * nf + ss * nc) * nlaunch;
    if (shifted)
      launch(STS_K_MG_UP, post, mg3_post_kernel<true, B, S, kPostT>, dim3(blocks), dim3(kPostT), 0,
             st, a);
    else
      launch(STS_K_MG_UP, post, mg3_post_kernel<false, B, S, kPostT>, dim3(blocks), dim3(kPostT), 0,
             st, a);
    STS_HIP(hipGetLastError());
  } else {
    const double post1 = ((sb + 3.0 * ss) * nf + ss * nc) * nlaunch;
    const double post2 = (2.0 * sb + 2.0 * ss) * nf * nlaunch;
    if (shifted)
      launch(STS_K_MG_UP, post1, mg3_post1_kernel<true, B, S>, dim3(blocks), dim3(kT), 0, st, a);
    else
      launch(STS_K_MG_UP, post1, mg3_post1_kernel<false, B, S>, dim3(blocks), dim3(kT), 0, st, a);
    STS_HIP(hipGetLastError());
    if (shifted)
      launch(STS_K_MG_UP, post2, mg3_post2_kernel<true, B, S>, dim3(blocks), dim3(kT), 0, st, a);
    else
      launch(STS_K_MG_UP, post2, mg3_post2_kernel<false, B, S>, dim3(blocks), dim3(kT), 0, st, a);
    STS_HIP(hipGetLastError());
  }
}

template <class T>
void coarse_solve(Coarse3Args c, const void* b, void* e, void* t1, void* part, int nlaunch,
                  hipStream_t st) {
  const int m = c.m;
  const double by = 2.0 * sizeof(T) * std::pow((double)m, 3) * nlaunch;
  const dim3 grid(m, nlaunch);
  c.in = b;
  c.out = t1;
  launch(STS_K_MG_COARSE, by, coarse3_plane_kernel<T>, grid, dim3(kCT), 0, st, c);
  STS_HIP(hipGetLastError());
  launch(STS_K_MG_COARSE, by, coarse3_z_kernel<T>, grid, dim3(kCT), 0, st, c);
  STS_HIP(hipGetLastError());
  c.in = t1;
  c.out = e;
  c.rhs = b;
  c.part = static_cast<double*>(part);
  launch(STS_K_MG_COARSE, by, coarse3_plane_kernel<T>, grid, dim3(kCT), 0, st, c);
  STS_HIP(hipGetLastError());
}

}  // namespace

void mg3_vcycle(const MGWork& w, const CGScal* act, const int* cols, int nlaunch, bool partials,
                hipStream_t st) {
  const MGPlan& p = w.plan;
  const int L = p.nlev;
  const Smooth sm = smooth_coefficients(kSmoothLo);
  const bool shifted = p.sw0 != 0.0;
  // the mixed-precision V-cycle needs a smoothed level: its finest vectors
  // (the PCG residual and preconditioned residual) stay FP64
  const bool f32 = (p.f32 || p.f32cg) && L > 0;
  // the FP32 PCG: its residual and preconditioned residual are FP32 as well
  const bool all32 = p.f32cg && L > 0;
  auto level = [&](int l) {
    Level3Args a{};
    a.nf = p.n[l];
    a.nc = p.n[l + 1];
    a.ldf = w.ld[l];
    a.ldc = w.ld[l + 1];
    a.bf = w.b[l];
    a.xp = w.xp[l];
    a.bc = w.b[l + 1];
    a.ec = w.e[l + 1];
    a.u1 = w.u1[l];
    a.d0 = w.d0[l];
    a.ef = w.e[l];
    a.nlaunch = nlaunch;
    for (int j = 0; j < nlaunch; ++j) a.cols[j] = cols[j];
    a.st = act;
    a.c = level_coef(p, l);
    a.sm = std::ldexp(p.sw0, 3 * l);   // (h_l / 6)^3 = 8^l (h / 6)^3
    a.a1 = sm.a[1];
    a.c0 = sm.c[0];
    a.c1 = sm.c[1];
    a.max_tiles = w.max_tiles;
    return a;
  };
  for (int l = 0; l < L; ++l) {
    if (!f32) level_down<double, double>(level(l), shifted, nlaunch, st);
    else if (l == 0 && !all32) level_down<double, float>(level(l), shifted, nlaunch, st);
    else level_down<float, float>(level(l), shifted, nlaunch, st);
  }
  {
    Coarse3Args c{};
    c.m = p.exact;
    c.ld = w.ld[L];
    c.dst = w.dst;
    c.c = level_coef(p, L);
    c.sm = std::ldexp(p.sw0, 3 * L);
    c.nlaunch = nlaunch;
    for (int j = 0; j < nlaunch; ++j) c.cols[j] = cols[j];
    c.st = act;
    c.max_tiles = w.max_tiles;
    void* part = (partials && L == 0) ? w.part_rz : nullptr;
    if (f32) coarse_solve<float>(c, w.b[L], w.e[L], w.t1, part, nlaunch, st);
    else coarse_solve<double>(c, w.b[L], w.e[L], w.t1, part, nlaunch, st);
  }
  for (int l = L - 1; l >= 0; --l) {
    Level3Args a = level(l);
    a.part = (partials && l == 0) ? w.part_rz : nullptr;
    if (!f32) level_up<double, double>(a, shifted, nlaunch, st);
    else if (l == 0 && !all32) level_up<double, float>(a, shifted, nlaunch, st);
    else level_up<float, float>(a, shifted, nlaunch, st);
  }
}

void pcg3_setup(const MGWork& w, const double* const* b, const int* cols, int nlaunch, int ncols,
                double rtol, int maxit, hipStream_t st) {
  PCG3Args a = pcg3_args(w, 0, cols, nlaunch, ncols);
  for (int j = 0; j < nlaunch; ++j) a.b[j] = b[j];
  for (int c = 0; c < kMaxCols; ++c) {
    const double rt = (w.col_rtol && c < ncols) ? w.col_rtol[c] : rtol;
    a.rtol2[c] = rt * rt;
  }
  const dim3 grid(a.ntx * a.nty * a.ntz * nlaunch);
  if (w.plan.f32cg && w.plan.x64)
    launch(STS_K_PCG_B, 16.0 * std::pow((double)a.n, 3) * nlaunch,
           pcg3_setup_kernel<float, double>, grid, dim3(kT), 0, st, a, maxit);
  else if (w.plan.f32cg)
    launch(STS_K_PCG_B, 12.0 * std::pow((double)a.n, 3) * nlaunch,
           pcg3_setup_kernel<float, float>, grid, dim3(kT), 0, st, a, maxit);
  else
    launch(STS_K_PCG_B, 40.0 * std::pow((double)a.n, 3) * nlaunch,
           pcg3_setup_kernel<double, double>, grid, dim3(kT), 0, st, a, maxit);
  STS_HIP(hipGetLastError());
}

void pcg3_iterate(const MGWork& w, int parity, const int* cols, int nlaunch, int ncols,
                  hipStream_t st) {
  mg3_vcycle(w, w.scal + (parity ^ 1) * kMaxCols, cols, nlaunch, true, st);
  PCG3Args a = pcg3_args(w, parity, cols, nlaunch, ncols);
  const int ntiles = a.ntx * a.nty * a.ntz;
  const int blocks = ntiles * nlaunch;
  const double nn = std::pow((double)a.n, 3) * nlaunch;
  const bool split = ntiles > kSplitReduceTiles;
  Reduce3Args r{};
  r.max_tiles = w.max_tiles;
  for (int j = 0; j < nlaunch; ++j) r.cols[j] = cols[j];
  if (split) {
    // (r, r) from the previous B (or the set-up), (r, z) from this V-cycle
    r.part[0] = w.part_rr;
    r.count[0] = ntiles;
    r.out[0] = w.tot;
    r.part[1] = w.part_rz;
    r.count[1] = a.rz_tiles;
    r.out[1] = w.tot + kMaxCols;
    launch(STS_K_PCG_REDUCE, 8.0 * (ntiles + a.rz_tiles) * nlaunch, pcg3_reduce_kernel,
           dim3(nlaunch, 2), dim3(kT), 0, st, r);
    STS_HIP(hipGetLastError());
    a.tot = w.tot;
  }
  const double vb = w.plan.f32cg ? 4.0 : 8.0;   // bytes per vector element
  if (w.plan.f32cg) {
    if (w.plan.sw0 != 0.0)
      launch(STS_K_PCG_A, 4.0 * vb * nn, pcg3_a_kernel<true, float>, dim3(blocks), dim3(kT), 0, st, a);
    else
      launch(STS_K_PCG_A, 4.0 * vb * nn, pcg3_a_kernel<false, float>, dim3(blocks), dim3(kT), 0, st, a);
  } else {
    if (w.plan.sw0 != 0.0)
      launch(STS_K_PCG_A, 4.0 * vb * nn, pcg3_a_kernel<true, double>, dim3(blocks), dim3(kT), 0, st, a);
    else
      launch(STS_K_PCG_A, 4.0 * vb * nn, pcg3_a_kernel<false, double>, dim3(blocks), dim3(kT), 0, st, a);
  }
  STS_HIP(hipGetLastError());
  if (split) {
    r.part[0] = w.part_pq;
    r.count[0] = ntiles;
    r.out[0] = w.tot + 2 * kMaxCols;
    launch(STS_K_PCG_REDUCE, 8.0 * ntiles * nlaunch, pcg3_reduce_kernel, dim3(nlaunch, 1),
           dim3(kT), 0, st, r);
    STS_HIP(hipGetLastError());
  }
  if (w.plan.f32cg && w.plan.x64)
    launch(STS_K_PCG_B, (4.0 * vb + 16.0) * nn, pcg3_b_kernel<float, double>, dim3(blocks),
           dim3(kT), 0, st, a);
  else if (w.plan.f32cg)
    launch(STS_K_PCG_B, 6.0 * vb * nn, pcg3_b_kernel<float, float>, dim3(blocks), dim3(kT), 0, st,
           a);
  else
    launch(STS_K_PCG_B, 6.0 * vb * nn, pcg3_b_kernel<double, double>, dim3(blocks), dim3(kT), 0,
           st, a);
  STS_HIP(hipGetLastError());
}

void mg3_defect(const MGWork& w, int ncols, double* const* x, const void* const* d, bool d32,
                const double* const* b, double* const* r, double* norms2, hipStream_t st) {
  Defect3Args a{};
  a.n = w.plan.n[0];
  a.ntx = (a.n + TX - 1) / TX;
  a.nty = (a.n + TY - 1) / TY;
  a.ntz = (a.n + TZ - 1) / TZ;
  a.nlaunch = ncols;
  bool any_d = false;
  for (int j = 0; j < ncols; ++j) {
    a.x[j] = x[j];
    a.d[j] = d ? d[j] : nullptr;
    a.b[j] = b[j];
    a.r[j] = r[j];
    any_d |= a.d[j] != nullptr;
  }
  a.c = w.plan.mu;
  a.sm = w.plan.sw0;
  a.part = w.part_rr;
  a.max_tiles = w.max_tiles;
  const int ntiles = a.ntx * a.nty * a.ntz;
  const int64_t nodes = (int64_t)a.n * a.n * a.n;
  const double nn = (double)nodes * ncols;
  if (any_d) {
    const dim3 ag((unsigned)std::min<int64_t>((nodes + kT - 1) / kT, 4096), (unsigned)ncols);
    if (d32)
      launch(STS_K_STENCIL, 20.0 * nn, add_corr3_kernel<float>, ag, dim3(kT), 0, st, a, nodes);
    else
      launch(STS_K_STENCIL, 24.0 * nn, add_corr3_kernel<double>, ag, dim3(kT), 0, st, a, nodes);
    STS_HIP(hipGetLastError());
  }
  const dim3 grid(ntiles * ncols);
  if (a.sm != 0.0)
    launch(STS_K_STENCIL, 24.0 * nn, defect3_kernel<true>, grid, dim3(kT), 0, st, a);
  else
    launch(STS_K_STENCIL, 24.0 * nn, defect3_kernel<false>, grid, dim3(kT), 0, st, a);
  STS_HIP(hipGetLastError());
  Reduce3Args rd{};
  rd.max_tiles = w.max_tiles;
  for (int j = 0; j < ncols; ++j) rd.cols[j] = j;
  rd.part[0] = w.part_rr;
  rd.count[0] = ntiles;
  rd.out[0] = norms2;
  launch(STS_K_PCG_REDUCE, 8.0 * ntiles * ncols, pcg3_reduce_kernel, dim3(ncols, 1), dim3(kT), 0,
         st, rd);
  STS_HIP(hipGetLastError());
}

void mg3_replace(const MGWork& w, const int* cols, int nl, hipStream_t st) {
  if (nl <= 0) return;
  Replace3Args a{};
  a.n = w.plan.n[0];
  a.ld = w.ld[0];
  a.ldx = w.ldx;
  a.ntx = (a.n + TX - 1) / TX;
  a.nty = (a.n + TY - 1) / TY;
  a.ntz = (a.n + TZ - 1) / TZ;
  a.nlaunch = nl;
  for (int j = 0; j < nl; ++j) a.cols[j] = cols[j];
  for (int c = 0; c < kMaxCols; ++c) a.b[c] = w.rhs[c];
  a.c = w.plan.mu;
  a.sm = w.plan.sw0;
  a.x = w.x;
  a.r = reinterpret_cast<float*>(w.b[0]);
  a.part = w.part_rr;
  a.max_tiles = w.max_tiles;
  const int ntiles = a.ntx * a.nty * a.ntz;
  const double by = 20.0 * std::pow((double)a.n, 3) * nl;
  if (a.sm != 0.0)
    launch(STS_K_PCG_A, by, replace3_kernel<true>, dim3(ntiles * nl), dim3(kT), 0, st, a);
  else
    launch(STS_K_PCG_A, by, replace3_kernel<false>, dim3(ntiles * nl), dim3(kT), 0, st, a);
  STS_HIP(hipGetLastError());
}

}  // namespace sts
