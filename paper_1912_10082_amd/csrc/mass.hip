// Mass-matrix solves Mx x = b by Chebyshev iteration (2-D P1).
//
// The expansion of the extended Krylov space (Sec. 4) applies Mx^{-1} to the
// positive-power columns and to F1.  For the P1 mass matrix of the uniform
// Courant triangulation, w (6; 1 at E, W, N, S, NE, SW) with w = h^2 / 12, the
// diagonal is D = 6 w and the spectrum of D^{-1} Mx lies in [1/2, 2] (the
// range of (6 + 2 cos a + 2 cos b + 2 cos(a + b)) / 6; Dirichlet sections
// stay inside it).  Chebyshev iteration for that interval needs no inner
// products, and its residual obeys ||r_k|| <= 2 q^k ||b|| with
// q = (sqrt(4) - 1) / (sqrt(4) + 1) = 1/3, so the iteration count follows from
// the tolerance alone.  Without reductions the steps can be fused: each
// launch runs up to kMassSteps steps on an LDS tile with a halo of that depth
// (the valid region shrinks by one node per step), so a solve is a handful of
// launches and never waits for the host.
#include <hip/hip_runtime.h>

#include <cmath>

#include "mg_common.h"
#include "sts_internal.h"

namespace sts {

namespace {

using mgc::ld_or_zero;
using mgc::StagedN;

constexpr int kT = 256;
constexpr int TX = 64, TY = 16;      // owned nodes per tile
constexpr int kS = kMassSteps;       // halo = most steps per launch
constexpr int W = TX + 2 * kS, H = TY + 2 * kS;

__device__ __forceinline__ int xcd_remap(int bid, int n) {
  const int q = n >> 3, rem = n & 7;
  const int x = bid & 7, j = bid >> 3;
  return x * q + min(x, rem) + j;
}

// Mx s / w at q (row width W): 6 s + E + W + N + S + NE + SW.
__device__ __forceinline__ double m7(const double* s, int q) {
  return 6.0 * s[q] + ((s[q - 1] + s[q + 1]) + (s[q - W] + s[q + W])) +
         (s[q + W + 1] + s[q - W - 1]);
}

struct MassArgs {
  int n;
  int ntx, nty;
  int nlaunch;
  int cols[kMaxCols];
  const double* b[kMaxCols];   // right-hand side of column cols[j], indexed by column
  const double* xin;           // state of the previous launch (stride ld), unused if k0 == 0
  const double* din;
  double* xout;                // state for the next launch, or the result
  double* dout;                // null on the last launch
  int64_t ld;                  // stride of xin / din / dout
  int64_t ldx;                 // stride of xout
  int k0, steps;               // first global step of this launch, steps in it
  double w;                    // h^2 / 12
  double a[kMassMaxIters];     // d_k = a_k d_{k-1} + c_k r_k / D
  double c[kMassMaxIters];
};

__global__ __launch_bounds__(kT) void mass_cheb_kernel(MassArgs a) {
  __shared__ double bs[W * H];
  __shared__ double xs[2][W * H];
  __shared__ double ds[W * H];
  const int ntiles = a.ntx * a.nty;
  const int lin = xcd_remap(blockIdx.x, a.nlaunch * ntiles);
  const int t = lin / a.nlaunch, col = a.cols[lin % a.nlaunch];
  const int n = a.n;
  const int x0 = (t % a.ntx) * TX - kS, y0 = (t / a.ntx) * TY - kS;
  const double* bg = a.b[col];
  const double inv_d = 1.0 / (6.0 * a.w);
  const bool fresh = a.k0 == 0;
  const double* xg = fresh ? nullptr : a.xin + (size_t)col * a.ld;
  const double* dg = fresh ? nullptr : a.din + (size_t)col * a.ld;
  {
    // all of a thread's loads in flight before the first LDS store
    auto at = [&](const double* v, int i) {
      const int gx = x0 + i % W, gy = y0 + i / W;
      return ld_or_zero(v, gx >= 0 && gx < n && gy >= 0 && gy < n, (size_t)gy * n + gx);
    };
    StagedN<W * H, double, kT> hb, hx, hd;
    hb.load([&](int i) { return at(bg, i); });
    if (!fresh) {
      hx.load([&](int i) { return at(xg, i); });
      hd.load([&](int i) { return at(dg, i); });
    }
    hb.store(bs);
    if (fresh) {
      for (int i = threadIdx.x; i < W * H; i += kT) {
        xs[0][i] = 0.0;
        xs[1][i] = 0.0;
        ds[i] = 0.0;
      }
    } else {
      hx.store(xs[0]);
      hx.store(xs[1]);
      hd.store(ds);
    }
  }
  __syncthreads();
  int cur = 0;
  for (int j = 0; j < a.steps; ++j) {
    const int k = a.k0 + j;
    const int sh = j + 1;   // valid region after this step
    const double ak = a.a[k], ck = a.c[k];
    for (int i = threadIdx.x; i < W * H; i += kT) {
      const int lx = i % W, ly = i / W;
      const int gx = x0 + lx, gy = y0 + ly;
      if (lx >= sh && lx < W - sh && ly >= sh && ly < H - sh && gx >= 0 && gx < n && gy >= 0 &&
          gy < n) {
        const double r = bs[i] - a.w * m7(xs[cur], i);
        const double d = ak * ds[i] + ck * inv_d * r;
        ds[i] = d;
        xs[cur ^ 1][i] = xs[cur][i] + d;
      }
    }
    __syncthreads();
    cur ^= 1;
  }
  // owned nodes
  double* xo = a.xout + (size_t)col * a.ldx;
  double* dout = a.dout ? a.dout + (size_t)col * a.ld : nullptr;
  for (int i = threadIdx.x; i < TX * TY; i += kT) {
    const int gx = x0 + kS + i % TX, gy = y0 + kS + i / TX;
    if (gx < n && gy < n) {
      const int q = (i / TX + kS) * W + (i % TX + kS);
      const size_t g = (size_t)gy * n + gx;
      xo[g] = xs[cur][q];
      if (dout) dout[g] = ds[q];
    }
  }
}

}  // namespace

int mass_cheb_iters(double rtol) {
  // ||r_k|| / ||b|| <= 2 q^k, q = 1/3
  const double k = std::log(rtol / 2.0) / std::log(1.0 / 3.0);
  return std::max(1, std::min(kMassMaxIters, (int)std::ceil(k)));
}

bool mass_cheb_supported(const Grid& g, const Stencil& M) {
  if (g.dim != 2 || g.nx != g.ny) return false;
  const double w = M.c[13] / 6.0;
  if (!(w > 0.0)) return false;
  for (int i = 0; i < 27; ++i) {
    double want = 0.0;
    if (i == 13) want = 6.0 * w;
    // E, W, N, S, NE, SW in the (dz+1)*9 + (dy+1)*3 + (dx+1) numbering
    if (i == 14 || i == 12 || i == 16 || i == 10 || i == 17 || i == 9) want = w;
    if (std::fabs(M.c[i] - want) > 1e-15 * std::fabs(w) * 8.0) return false;
  }
  return true;
}

void mass_cheb_solve(const Grid& g, const Stencil& M, int ncols, const double* const* b,
                     double* x, int64_t ldx, double* xbuf[2], double* dbuf[2], int64_t ld,
                     int iters, hipStream_t st) {
  STS_REQUIRE(ncols >= 1 && ncols <= kMaxCols, STS_E_INVALID, "mass solve: 1..8 columns");
  STS_REQUIRE(iters >= 1 && iters <= kMassMaxIters, STS_E_INVALID, "mass solve: iterations");
  MassArgs a{};
  a.n = g.nx;
  a.ntx = (g.nx + TX - 1) / TX;
  a.nty = (g.nx + TY - 1) / TY;
  a.nlaunch = ncols;
  for (int c = 0; c < ncols; ++c) {
    a.cols[c] = c;
    a.b[c] = b[c];
  }
  a.ld = ld;
  a.w = M.c[13] / 6.0;
  // Chebyshev coefficients for [1/2, 2]
  const double lo = 0.5, hi = 2.0;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  double rho = 1.0 / sigma;
  a.a[0] = 0.0;
  a.c[0] = 1.0 / theta;
  for (int k = 1; k < iters; ++k) {
    const double rho1 = 1.0 / (2.0 * sigma - rho);
    a.a[k] = rho1 * rho;
    a.c[k] = 2.0 * rho1 / delta;
    rho = rho1;
  }
  const int nl = (iters + kS - 1) / kS;
  const int blocks = a.ntx * a.nty * ncols;
  int k0 = 0;
  for (int l = 0; l < nl; ++l) {
    const int steps = (iters - k0 + (nl - l) - 1) / (nl - l);   // spread evenly
    a.k0 = k0;
    a.steps = steps;
    a.xin = xbuf[(l + 1) & 1];
    a.din = dbuf[(l + 1) & 1];
    const bool last = l == nl - 1;
    a.xout = last ? x : xbuf[l & 1];
    a.ldx = last ? ldx : ld;
    a.dout = last ? nullptr : dbuf[l & 1];
    // read b (and x, d after the first launch), write x (and d before the last)
    const double per = 8.0 + (k0 == 0 ? 0.0 : 16.0) + 8.0 + (last ? 0.0 : 8.0);
    launch(STS_K_MASS_CHEB, per * g.nh * ncols, mass_cheb_kernel, dim3(blocks), dim3(kT), 0, st, a);
    STS_HIP(hipGetLastError());
    k0 += steps;
  }
}

}  // namespace sts
