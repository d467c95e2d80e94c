// Symmetric eigendecomposition of the reduced matrix Km (Sec. 4: the reduced
// spatial pencil is diagonalised before the time sweep).
//
// Stages (each its own launch):
//  1. tridiag_kernel: Householder reduction to tridiagonal form in one
//     work-group, blocked by panels of kNB columns: inside a panel each
//     reflector's symmetric matrix-vector product reads the trailing matrix
//     as of the panel start and corrects for the panel's earlier reflectors
//     with their images W (y = A v - V (W^T v) - W (V^T v)); the rank-2 kNB
//     update of the trailing matrix is applied once per panel.
//  2. bisect_kernel: eigenvalues of the tridiagonal T by multisection of the
//     Sturm count, kSect threads per eigenvalue, many work-groups.
//  3. inviter_kernel: eigenvectors of T by inverse iteration, one thread per
//     eigenvalue (LU with partial pivoting of T - lambda I, three solves from
//     a pseudo-random start).  Eigenvalues closer than kClusterTol ||T|| form
//     a cluster, handled by one thread that orthogonalises each member
//     against the earlier ones after every solve.
//  4. Orthogonalisation: inverse-iteration vectors of eigenvalues a gap g
//     apart are orthogonal only to about eps ||T|| / g.  Two Newton-Schulz
//     steps Z <- Z (3 I - Z^T Z) / 2 (matrix-core GEMMs) make Z orthonormal to
//     rounding; the mixing they introduce between two eigenvectors is of the
//     order eps ||T|| / g, so it changes the residual by about eps ||T|| and
//     the decomposition stays backward stable.  Eigenvalues are the Rayleigh
//     quotients z_j^T T z_j.
//  5. backtransform_kernel: Q = H_0 H_1 ... H_{k-3} Z, one wave per column.
#include <hip/hip_runtime.h>

#include <cmath>

#include "sts_internal.h"

namespace sts {

namespace {

constexpr int kTT = 1024;            // threads of the tridiagonalisation work-group
constexpr int kSect = 4;             // threads per eigenvalue in the multisection
constexpr double kEps = 1.1102230246251565e-16;
// Inverse iteration from a shift within ~eps ||T|| of its eigenvalue leaves
// an overlap near eps ||T|| / g with an eigenvector g away; down to gaps of
// 1e-11 ||T|| that is <= 1e-5, which the two Newton-Schulz steps remove
// (1e-5 -> 1e-10 -> rounding).  Closer eigenvalues are a cluster.  A wider
// tolerance made the graded spectra of 1-D reduced matrices (||T|| ~ 1e10,
// gaps ~ 1 among the small Ritz values) one sequential cluster of dozens.
constexpr double kClusterTol = 1e-11;
constexpr int kInvIters = 3;
constexpr int kLdsPanelMaxK = 480;   // orders whose tridiagonalisation panel fits in LDS

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the 1024-thread work-group, fixed order; result broadcast.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < kTT / 64; ++i) t += red[i];
  return t;
}

// ---------------------------------------------------------------------------
// 1. tridiagonalisation
// ---------------------------------------------------------------------------
struct TriArgs {
  int k;
  const double* A;
  int64_t lda;
  int* status;
  double* a;        // k x k, ld k
  double* d;
  double* e;
  double* tau;
  double* vp;       // k x kEigNB
  double* wp;       // k x kEigNB
  double* bounds;   // gl, gu, tnorm, pivmin
};

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64: lane l = i + 16 g supplies a = X[i][g] and
// b = Y[g][i]; element q of the accumulator is (X Y)[4 q + g][i].
__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// LP: the panel's reflectors V and images W live in LDS (orders up to
// kLdsPanelMaxK), else in global scratch.
template <bool LP>
__global__ __launch_bounds__(kTT) void tridiag_kernel(TriArgs g) {
  constexpr int VK = LP ? kLdsPanelMaxK : kEigMaxK;
  __shared__ double v[VK];
  __shared__ double y[VK];
  __shared__ double cj[VK];
  __shared__ double part[kTT];
  __shared__ double red[kTT / 64];
  __shared__ double t12[2 * kEigNB];
  __shared__ double panel[LP ? 2 * kLdsPanelMaxK * kEigNB : 1];
  const int k = g.k;
  const int tid = threadIdx.x;
  double* a = g.a;
  double* vp = LP ? panel : g.vp;
  double* wp = LP ? panel + kLdsPanelMaxK * kEigNB : g.wp;
  const int ldp = LP ? kLdsPanelMaxK : k;

  double fin = 0.0;
  for (int64_t idx = tid; idx < (int64_t)k * k; idx += kTT) {
    const int i = idx % k, j = idx / k;
    const double x = 0.5 * (g.A[i + j * g.lda] + g.A[j + i * g.lda]);
    a[idx] = x;
    fin += x * 0.0;   // NaN if any entry is not finite
  }
  fin = block_sum(fin, red);
  if (tid == 0) *g.status = fin == 0.0 ? 0 : 1;
  if (fin != 0.0) return;   // uniform: every thread holds the same sum

  for (int j0 = 0; j0 + 2 < k; j0 += kEigNB) {
    const int jb = min(kEigNB, k - 2 - j0);
    for (int jj = 0; jj < jb; ++jj) {
      const int j = j0 + jj;
      const int n2 = k - j - 1;
      double* col = a + (int64_t)j * k;
      // column j (rows j..k-1) with the panel's earlier reflectors applied,
      // and the squared norm below row j+1
      double sq = 0.0;
      for (int i = j + tid; i < k; i += kTT) {
        double s = col[i];
        for (int q = 0; q < jj; ++q)
          s -= vp[i + q * ldp] * wp[j + q * ldp] + wp[i + q * ldp] * vp[j + q * ldp];
        cj[i] = s;
        if (i >= j + 2) sq += s * s;
      }
      const double sig = block_sum(sq, red);
      const double alpha = cj[j + 1];
      double tau = 0.0, beta = alpha, scale = 0.0;
      if (sig > 0.0) {
        const double nrm = sqrt(alpha * alpha + sig);
        beta = alpha <= 0.0 ? nrm : -nrm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      // reflector v (v_0 = 1), kept below the sub-diagonal of column j
      for (int i = tid; i < n2; i += kTT) {
        const double vi = (i == 0) ? 1.0 : cj[j + 1 + i] * scale;
        v[i] = vi;
        if (i > 0) col[j + 1 + i] = vi;
      }
      if (tid == 0) {
        g.d[j] = cj[j];
        g.e[j] = beta;
        g.tau[j] = tau;
      }
      __syncthreads();
      if (tau == 0.0) {
        for (int i = tid; i < n2; i += kTT) {
          vp[j + 1 + i + jj * ldp] = 0.0;
          wp[j + 1 + i + jj * ldp] = 0.0;
        }
        __syncthreads();
        continue;
      }
      // t1 = W_p^T v, t2 = V_p^T v over rows j+1..k-1 (one wave per product)
      {
        const int wv = tid >> 6, lane = tid & 63;
        for (int q = wv; q < 2 * jj; q += kTT / 64) {
          const double* src = (q < jj ? wp : vp) + (q % jj) * ldp + (j + 1);
          double s = 0.0;
          for (int i = lane; i < n2; i += 64) s += src[i] * v[i];
          s = wave_sum(s);
          if (lane == 0) t12[q] = s;
        }
      }
      // y = A22 v, A22 = a[j+1.., j+1..] as of the panel start
      const double* A22 = a + (j + 1) + (int64_t)(j + 1) * k;
      for (int base = 0; base < n2; base += kTT / 4) {
        const int r = base + (tid & (kTT / 4 - 1));
        const int pq = tid / (kTT / 4);
        double s = 0.0;
        if (r < n2) {
          const int c0 = (n2 * pq) / 4, c1 = (n2 * (pq + 1)) / 4;
          // four independent chains keep four loads of the column sweep in
          // flight (7% faster than one chain at k = 228)
          double s1 = 0.0, s2 = 0.0, s3 = 0.0;
          int c = c0;
          for (; c + 4 <= c1; c += 4) {
            s += A22[r + (int64_t)c * k] * v[c];
            s1 += A22[r + (int64_t)(c + 1) * k] * v[c + 1];
            s2 += A22[r + (int64_t)(c + 2) * k] * v[c + 2];
            s3 += A22[r + (int64_t)(c + 3) * k] * v[c + 3];
          }
          for (; c < c1; ++c) s += A22[r + (int64_t)c * k] * v[c];
          s = (s + s1) + (s2 + s3);
        }
        part[tid] = s;
        __syncthreads();
        if (pq == 0 && r < n2) {
          const int q = tid & (kTT / 4 - 1);
          y[r] = (part[q] + part[q + kTT / 4]) + (part[q + kTT / 2] + part[q + 3 * kTT / 4]);
        }
        __syncthreads();
      }
      // p = tau (y - V_p t1 - W_p t2); w = p - (tau / 2)(p . v) v
      double pv = 0.0;
      for (int i = tid; i < n2; i += kTT) {
        double s = y[i];
        for (int q = 0; q < jj; ++q)
          s -= vp[j + 1 + i + q * ldp] * t12[q] + wp[j + 1 + i + q * ldp] * t12[jj + q];
        s *= tau;
        y[i] = s;
        pv += s * v[i];
      }
      pv = block_sum(pv, red);
      const double kk = -0.5 * tau * pv;
      for (int i = tid; i < n2; i += kTT) {
        vp[j + 1 + i + jj * ldp] = v[i];
        wp[j + 1 + i + jj * ldp] = y[i] + kk * v[i];
      }
      __syncthreads();
    }
    // trailing update A[t0.., t0..] -= [V W] [W V]^T on the matrix cores,
    // one 16 x 16 tile per wave at a time
    const int t0 = j0 + jb;
    const int nt2 = k - t0;
    const int tiles = (nt2 + 15) / 16;
    const int lane = tid & 63, wv = tid >> 6, li = lane & 15, lg = lane >> 4;
    for (int tt = wv; tt < tiles * tiles; tt += kTT / 64) {
      const int r0 = t0 + (tt % tiles) * 16, c0 = t0 + (tt / tiles) * 16;
      const int r = r0 + li, c = c0 + li;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < 2 * jb; k0 += 4) {
        const int q = k0 + lg;
        double xa = 0.0, yb = 0.0;
        if (q < 2 * jb) {
          if (r < k) xa = q < jb ? vp[r + q * ldp] : wp[r + (q - jb) * ldp];
          if (c < k) yb = q < jb ? wp[c + q * ldp] : vp[c + (q - jb) * ldp];
        }
        acc = mfma(xa, yb, acc);
      }
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int rr = r0 + 4 * qq + lg;
        if (rr < k && c < k) a[rr + (int64_t)c * k] -= acc[qq];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (k >= 2) {
      g.d[k - 2] = a[(k - 2) + (int64_t)(k - 2) * k];
      g.e[k - 2] = a[(k - 1) + (int64_t)(k - 2) * k];
    }
    g.d[k - 1] = a[(k - 1) + (int64_t)(k - 1) * k];
    g.e[k - 1] = 0.0;
  }
  __syncthreads();
  // Gershgorin interval, ||T||, and the smallest pivot of the Sturm counts
  double lo = 1e308, hi = -1e308, emax = 0.0;
  for (int i = tid; i < k; i += kTT) {
    const double r = (i > 0 ? fabs(g.e[i - 1]) : 0.0) + (i + 1 < k ? fabs(g.e[i]) : 0.0);
    lo = fmin(lo, g.d[i] - r);
    hi = fmax(hi, g.d[i] + r);
    if (i + 1 < k) emax = fmax(emax, g.e[i] * g.e[i]);
  }
  // min / max reductions through the partial array
  part[tid] = lo;
  __syncthreads();
  for (int s = kTT / 2; s > 0; s >>= 1) {
    if (tid < s) part[tid] = fmin(part[tid], part[tid + s]);
    __syncthreads();
  }
  lo = part[0];
  __syncthreads();
  part[tid] = hi;
  __syncthreads();
  for (int s = kTT / 2; s > 0; s >>= 1) {
    if (tid < s) part[tid] = fmax(part[tid], part[tid + s]);
    __syncthreads();
  }
  hi = part[0];
  __syncthreads();
  part[tid] = emax;
  __syncthreads();
  for (int s = kTT / 2; s > 0; s >>= 1) {
    if (tid < s) part[tid] = fmax(part[tid], part[tid + s]);
    __syncthreads();
  }
  if (tid == 0) {
    const double tnorm = fmax(fmax(fabs(lo), fabs(hi)), 2.2250738585072014e-308);
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, part[0]);
    const double widen = (2.0 + k) * kEps * tnorm + 2.0 * pivmin;
    g.bounds[0] = lo - widen;
    g.bounds[1] = hi + widen;
    g.bounds[2] = tnorm;
    g.bounds[3] = pivmin;
  }
}

// ---------------------------------------------------------------------------
// 2. eigenvalues by multisection of the Sturm count
// ---------------------------------------------------------------------------

// Number of eigenvalues of T below x.
__device__ int sturm_count(const double* d, const double* e, int k, double x, double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
  for (int i = 1; i < k; ++i) {
    q = (d[i] - x) - e[i - 1] * e[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

__global__ __launch_bounds__(256) void bisect_kernel(int k, const double* d, const double* e,
                                                     const double* bounds, double* lam) {
  __shared__ double ds[kEigMaxK];
  __shared__ double es[kEigMaxK];
  for (int i = threadIdx.x; i < k; i += 256) {
    ds[i] = d[i];
    es[i] = i + 1 < k ? e[i] : 0.0;
  }
  __syncthreads();
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int j = t / kSect, s = t % kSect;
  const bool act = j < k;
  const double pivmin = bounds[3];
  double lo = bounds[0], hi = bounds[1];
  for (int it = 0; it < 64; ++it) {
    const double w = hi - lo;
    const bool done = !(w > 2.0 * kEps * fmax(fabs(lo), fabs(hi)) + pivmin);
    // the group of kSect lanes shares the decision; a converged group idles
    const double x = lo + w * (double)(s + 1) / (double)(kSect + 1);
    const int c = (act && !done) ? sturm_count(ds, es, k, x, pivmin) : 0;
    double nlo = lo, nhi = hi;
#pragma unroll
    for (int u = 0; u < kSect; ++u) {
      const int cu = __shfl(c, (threadIdx.x & ~(kSect - 1)) + u, 64);
      const double xu = lo + w * (double)(u + 1) / (double)(kSect + 1);
      if (cu <= j) nlo = fmax(nlo, xu);
      else nhi = fmin(nhi, xu);
    }
    if (!done) {
      lo = nlo;
      hi = nhi;
    }
    // every group of the wave finished: stop (uniform per wave)
    if (__all(done || !act)) break;
  }
  if (act && s == 0) lam[j] = 0.5 * (lo + hi);
}

// ---------------------------------------------------------------------------
// 3. inverse iteration
// ---------------------------------------------------------------------------

__device__ __forceinline__ double start_value(int i, int j) {
  unsigned x = (unsigned)i * 2654435761u ^ ((unsigned)j * 40503u + 0x9e3779b9u);
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return (double)(x & 0xffffff) / (double)0x800000 - 1.0;   // [-1, 1)
}

struct InvArgs {
  int k;
  const double* d;
  const double* e;
  const double* lam;
  const double* bounds;
  double* z;        // k x k, ld k
  double* lu;       // 5 k^2 (factor f, row i, thread j at (f k + i) k + j)
  double* xt;       // k^2: the iterate of thread j, row i at i k + j
};

// Steps of the triangular solves whose operands are loaded together: the
// solves are one dependent chain per thread, so each step's loads are issued
// a chunk ahead instead of in the chain.
constexpr int kInvChunk = 8;

__global__ __launch_bounds__(64) void inviter_kernel(InvArgs g) {
  const int j0 = blockIdx.x * 64 + threadIdx.x;
  const int k = g.k;
  if (j0 >= k) return;
  const double tnorm = g.bounds[2];
  const double ctol = kClusterTol * tnorm;
  // cluster leader: first eigenvalue of a run with gaps <= ctol
  if (j0 > 0 && g.lam[j0] - g.lam[j0 - 1] <= ctol) return;
  int m = 1;
  while (j0 + m < k && g.lam[j0 + m] - g.lam[j0 + m - 1] <= ctol) ++m;
  const double ptol = kEps * tnorm;   // smallest pivot magnitude
  double* u1 = g.lu;
  double* u2 = g.lu + (int64_t)k * k;
  double* u3 = g.lu + 2 * (int64_t)k * k;
  double* ml = g.lu + 3 * (int64_t)k * k;
  double* pv = g.lu + 4 * (int64_t)k * k;
  auto at = [&](double* base, int i) -> double& { return base[(int64_t)i * k + j0]; };
  double shift_prev = 0.0;
  for (int mm = 0; mm < m; ++mm) {
    const int j = j0 + mm;
    double shift = g.lam[j];
    if (mm > 0) {
      const double sep = 10.0 * kEps * fabs(shift);
      if (shift - shift_prev < sep) shift = shift_prev + sep;
    }
    shift_prev = shift;
    // LU with partial pivoting of T - shift I
    double cd = g.d[0] - shift, cs = k > 1 ? g.e[0] : 0.0;
    for (int i = 0; i + 1 < k; ++i) {
      const double c = g.e[i];
      const double an = g.d[i + 1] - shift;
      const double bn = (i + 2 < k) ? g.e[i + 1] : 0.0;
      if (fabs(cd) >= fabs(c)) {
        const double mult = cd != 0.0 ? c / cd : 0.0;
        at(u1, i) = cd;
        at(u2, i) = cs;
        at(u3, i) = 0.0;
        at(ml, i) = mult;
        at(pv, i) = 0.0;
        cd = an - mult * cs;
        cs = bn;
      } else {
        const double mult = cd / c;
        at(u1, i) = c;
        at(u2, i) = an;
        at(u3, i) = bn;
        at(ml, i) = mult;
        at(pv, i) = 1.0;
        cd = cs - mult * an;
        cs = -mult * bn;
      }
    }
    at(u1, k - 1) = cd;
    // pseudo-random start; the iterate is kept row-interleaved across the
    // threads (row i of thread j0 at xt[i k + j0]) for coalesced access
    auto x = [&](int i) -> double& { return g.xt[(int64_t)i * k + j0]; };
    for (int i = 0; i < k; ++i) x(i) = start_value(i, j);
    for (int it = 0; it < kInvIters; ++it) {
      // forward: row interchanges and L; the chain runs through `carry`
      // (the updated row i + 1)
      double carry = x(0);
      for (int i0 = 0; i0 + 1 < k; i0 += kInvChunk) {
        const int n = min(kInvChunk, k - 1 - i0);
        double xn[kInvChunk], mv[kInvChunk], pw[kInvChunk], out[kInvChunk];
#pragma unroll
        for (int c = 0; c < kInvChunk; ++c) {
          if (c < n) {
            xn[c] = x(i0 + c + 1);
            mv[c] = at(ml, i0 + c);
            pw[c] = at(pv, i0 + c);
          }
        }
#pragma unroll
        for (int c = 0; c < kInvChunk; ++c) {
          if (c < n) {
            double xi = carry, xnn = xn[c];
            if (pw[c] != 0.0) {
              const double t = xi;
              xi = xnn;
              xnn = t;
            }
            out[c] = xi;
            carry = xnn - mv[c] * xi;
          }
        }
#pragma unroll
        for (int c = 0; c < kInvChunk; ++c)
          if (c < n) x(i0 + c) = out[c];
      }
      x(k - 1) = carry;
      // backward: U with two super-diagonals, tiny pivots perturbed
      double x1 = 0.0, x2 = 0.0;
      for (int i1 = k - 1; i1 >= 0; i1 -= kInvChunk) {
        const int n = min(kInvChunk, i1 + 1);
        double xv[kInvChunk], a1[kInvChunk], a2[kInvChunk], a3[kInvChunk];
#pragma unroll
        for (int c = 0; c < kInvChunk; ++c) {
          if (c < n) {
            const int i = i1 - c;
            xv[c] = x(i);
            a1[c] = at(u1, i);
            a2[c] = at(u2, i);
            a3[c] = at(u3, i);
          }
        }
#pragma unroll
        for (int c = 0; c < kInvChunk; ++c) {
          if (c < n) {
            double p = a1[c];
            if (fabs(p) < ptol) p = p < 0.0 ? -ptol : ptol;
            const double xi = (xv[c] - a2[c] * x1 - a3[c] * x2) / p;
            xv[c] = xi;
            x2 = x1;
            x1 = xi;
          }
        }
#pragma unroll
        for (int c = 0; c < kInvChunk; ++c)
          if (c < n) x(i1 - c) = xv[c];
      }
      // orthogonalise against the earlier members of the cluster
      for (int q = 0; q < mm; ++q) {
        const double* zq = g.z + (int64_t)(j0 + q) * k;
        double s = 0.0;
        for (int i = 0; i < k; ++i) s += zq[i] * x(i);
        for (int i = 0; i < k; ++i) x(i) -= s * zq[i];
      }
      // normalise (infinity norm between solves, 2-norm at the end)
      double nrm = 0.0;
      if (it + 1 < kInvIters) {
#pragma unroll 8
        for (int i = 0; i < k; ++i) nrm = fmax(nrm, fabs(x(i)));
      } else {
#pragma unroll 8
        for (int i = 0; i < k; ++i) nrm += x(i) * x(i);
        nrm = sqrt(nrm);
      }
      const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
#pragma unroll 8
      for (int i = 0; i < k; ++i) x(i) *= inv;
    }
    // the finished vector into column j of z
    double* zj = g.z + (int64_t)j * k;
    for (int i = 0; i < k; ++i) zj[i] = x(i);
  }
}

// ---------------------------------------------------------------------------
// 4. Rayleigh-Ritz correction helpers
// ---------------------------------------------------------------------------

// TZ = T Z for the tridiagonal (d, e) and Z (k x k, ld k).
__global__ void tz_kernel(int k, const double* d, const double* e, const double* z, double* tz) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)k * k) return;
  const int i = idx % k;
  double s = d[i] * z[idx];
  if (i > 0) s += e[i - 1] * z[idx - 1];
  if (i + 1 < k) s += e[i] * z[idx + 1];
  tz[idx] = s;
}

// C = (3 I - G) / 2: one Newton-Schulz step towards the orthogonal factor.
__global__ void ns_kernel(int k, const double* G, double* C) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)k * k) return;
  const int i = idx % k, j = idx / k;
  C[idx] = (i == j ? 1.5 : 0.0) - 0.5 * G[idx];
}

// lam_j = z_j^T (T z_j), one wave per column.
__global__ __launch_bounds__(256) void rayleigh_kernel(int k, const double* z, const double* tz,
                                                       double* lam) {
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (j >= k) return;
  double s = 0.0;
  for (int i = lane; i < k; i += 64) s += z[i + (int64_t)j * k] * tz[i + (int64_t)j * k];
  s = wave_sum(s);
  if (lane == 0) lam[j] = s;
}

// ---------------------------------------------------------------------------
// 5. back-transformation: Q[:, c] = H_0 ... H_{k-3} z_c, one wave per column
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void backtransform_kernel(int k, const double* a,
                                                            const double* tau, const double* z,
                                                            double* Q, int64_t ldq) {
  extern __shared__ double zs[];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + wv;
  if (c >= k) return;
  double* x = zs + (int64_t)wv * k;
  for (int i = lane; i < k; i += 64) x[i] = z[i + (int64_t)c * k];
  for (int j = k - 3; j >= 0; --j) {
    const double t = tau[j];
    if (t == 0.0) continue;
    const int n2 = k - j - 1;
    const double* vj = a + (j + 1) + (int64_t)j * k;   // v_0 = 1 implicit
    double s = 0.0;
    for (int i = lane; i < n2; i += 64) s += (i == 0 ? 1.0 : vj[i]) * x[j + 1 + i];
    s = t * wave_sum(s);
    for (int i = lane; i < n2; i += 64) x[j + 1 + i] -= s * (i == 0 ? 1.0 : vj[i]);
  }
  for (int i = lane; i < k; i += 64) Q[i + (int64_t)c * ldq] = x[i];
}

}  // namespace

int64_t eig_work_doubles(int k) {
  const int64_t kk = (int64_t)k * k;
  return kk                       // a
         + 4 * (int64_t)k          // d, e, tau, spare
         + 2 * (int64_t)k * kEigNB // vp, wp
         + 8                       // bounds
         + 4 * kk                  // z, T z / Newton-Schulz factor, Z^T Z, second z
         + 5 * kk;                 // inverse-iteration factors
}

void sym_eigvals(int k, const double* A, int64_t lda, double* lam, const EigWork& w,
                 hipStream_t st) {
  STS_REQUIRE(k >= 1 && k <= kEigMaxK, STS_E_INVALID, "sym_eigvals: order out of range");
  // the workspace layout of sym_eig, first two stages only
  const int64_t kk = (int64_t)k * k;
  double* p = w.base;
  double* a = p;
  p += kk;
  double* d = p;
  double* e = p + k;
  double* tau = p + 2 * k;
  p += 4 * (int64_t)k;
  double* vp = p;
  double* wp = p + (int64_t)k * kEigNB;
  p += 2 * (int64_t)k * kEigNB;
  double* bounds = p;
  TriArgs t{k, A, lda, w.status, a, d, e, tau, vp, wp, bounds};
  const double kk8 = 8.0 * (double)k * k;
  if (k <= kLdsPanelMaxK)
    launch(STS_K_TRIDIAG, kk8, tridiag_kernel<true>, dim3(1), dim3(kTT), 0, st, t);
  else
    launch(STS_K_TRIDIAG, kk8, tridiag_kernel<false>, dim3(1), dim3(kTT), 0, st, t);
  STS_HIP(hipGetLastError());
  const int nthreads = k * kSect;
  launch(STS_K_BISECT, 24.0 * k, bisect_kernel, dim3((nthreads + 255) / 256), dim3(256), 0, st, k,
         d, e, bounds, lam);
  STS_HIP(hipGetLastError());
}

void sym_eig(int k, const double* A, int64_t lda, double* lam, double* Q, int64_t ldq,
             const EigWork& w, hipStream_t st) {
  STS_REQUIRE(k >= 1 && k <= kEigMaxK, STS_E_INVALID, "sym_eig: order out of range");
  const int64_t kk = (int64_t)k * k;
  double* p = w.base;
  double* a = p;
  p += kk;
  double* d = p;
  double* e = p + k;
  double* tau = p + 2 * k;
  p += 4 * (int64_t)k;
  double* vp = p;
  double* wp = p + (int64_t)k * kEigNB;
  p += 2 * (int64_t)k * kEigNB;
  double* bounds = p;
  p += 8;
  double* z = p;
  double* tzc = p + kk;
  double* G = p + 2 * kk;
  double* B = p + 3 * kk;
  p += 4 * kk;
  double* lu = p;

  TriArgs t{k, A, lda, w.status, a, d, e, tau, vp, wp, bounds};
  const double kk8 = 8.0 * (double)k * k;
  if (k <= kLdsPanelMaxK)
    launch(STS_K_TRIDIAG, kk8, tridiag_kernel<true>, dim3(1), dim3(kTT), 0, st, t);
  else
    launch(STS_K_TRIDIAG, kk8, tridiag_kernel<false>, dim3(1), dim3(kTT), 0, st, t);
  STS_HIP(hipGetLastError());
  const int nthreads = k * kSect;
  launch(STS_K_BISECT, 24.0 * k, bisect_kernel, dim3((nthreads + 255) / 256), dim3(256), 0, st, k,
         d, e, bounds, lam);
  STS_HIP(hipGetLastError());
  InvArgs iv{k, d, e, lam, bounds, z, lu, B};   // B is free until the Newton-Schulz steps
  launch(STS_K_INVITER, kk8, inviter_kernel, dim3((k + 63) / 64), dim3(64), 0, st, iv);
  STS_HIP(hipGetLastError());
  // two Newton-Schulz steps Z <- Z (3 I - Z^T Z) / 2 (ping-pong z / B)
  const unsigned nb = (unsigned)((kk + 255) / 256);
  double* zc = z;
  double* zn = B;
  for (int step = 0; step < 2; ++step) {
    gemm_small(true, k, k, k, 1.0, zc, k, zc, k, 0.0, G, k, st);
    ns_kernel<<<nb, 256, 0, st>>>(k, G, tzc);
    STS_HIP(hipGetLastError());
    gemm_small(false, k, k, k, 1.0, zc, k, tzc, k, 0.0, zn, k, st);
    double* t = zc;
    zc = zn;
    zn = t;
  }
  tz_kernel<<<nb, 256, 0, st>>>(k, d, e, zc, tzc);
  STS_HIP(hipGetLastError());
  rayleigh_kernel<<<(k + 3) / 4, 256, 0, st>>>(k, zc, tzc, lam);
  STS_HIP(hipGetLastError());
  launch(STS_K_BACKTRANSFORM, 2.0 * kk8, backtransform_kernel, dim3((k + 3) / 4), dim3(256),
         (unsigned)(4 * (size_t)k * sizeof(double)), st, k, a, tau, zc, Q, ldq);
  STS_HIP(hipGetLastError());
}

}  // namespace sts
