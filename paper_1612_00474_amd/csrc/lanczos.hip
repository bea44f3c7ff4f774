// Krylov/Lanczos approximation of M^{1/2} w (paper, Sec. II.C, method of Ando et al.).
//
// Everything but the O(N^2) products is float64 and O(N m):
//   v_1 = w/|w|;  for m = 1, 2, ...:
//     u = M v_m;  alpha_m = v_m . u;  u -= alpha_m v_m + beta_{m-1} v_{m-1};
//     u -= V_m (V_m^T u)                       (full re-orthogonalisation)
//     beta_m = |u|
//     T_m = Q L Q^T (updated from T_{m-1}'s), y_m = |w| Q L^{1/2} Q^T e_1
//     eps_m = |y_m - (y_{m-1}, 0)| / |y_{m-1}|  (= |g_m - g_{m-1}|/|g_{m-1}| for orthonormal V)
//     stop if eps_m < tol (m >= 2), or beta_m ~ 0 (invariant Krylov space, exact result)
//     v_{m+1} = u / beta_m
//   g = V_m y_m.
// Reductions use a fixed number of blocks and a fixed tree, so results are bitwise
// reproducible.  The host reads a 32-byte status record once per iteration.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <condition_variable>
#include <cstddef>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "rpb_internal.h"

namespace rpb {

namespace {

constexpr int kMaxKrylov = 64;      // largest m (the eigensolve keeps T_m in one wavefront)
constexpr int kRedBlocks = 256;     // partial sums per reduction
constexpr int kThreads = 256;

// Device-side Lanczos scalars (lives at the start of the WS_SMALL slot).
struct LzState {
  double alpha[kMaxKrylov];
  double beta[kMaxKrylov];
  double y[kMaxKrylov];
  double yprev[kMaxKrylov];
  double h[kMaxKrylov];
  double wnorm;
  int halt;       // set by the vector work once it has seen reason != 0 (read by the products)
  int pad_;
  // status (read by the host every iteration)
  double eps;
  int m;
  int reason;     // 0 running, 1 converged, 2 breakdown, 3 not SPD, 4 eigensolve failed
};
static_assert(sizeof(LzState) % 8 == 0, "LzState is an array of doubles and pairs of ints");
static_assert(sizeof(LzState) <= kSmallWorkCounter, "LzState must fit the start of the small slot");
static_assert(size_t(kMaxBatchSystems) * sizeof(LzStatus) <= kHostLzRingOffset,
              "per-system records must stay below the status ring");

// Host copies of the status words (eps, m, reason) of consecutive iterations, slot k mod
// kLzRing for iteration k.
struct LzRingSlot {
  double eps;
  int m;
  int reason;
};
struct LzRing {
  LzRingSlot slot[kLzRing];
};
static_assert(sizeof(LzRingSlot) == sizeof(double) + 2 * sizeof(int) &&
                  offsetof(LzState, reason) - offsetof(LzState, eps) ==
                      offsetof(LzRingSlot, reason) - offsetof(LzRingSlot, eps),
              "the ring slot mirrors the status words of LzState");

LzRing *lz_ring(rpb_ctx *ctx) {
  return reinterpret_cast<LzRing *>(static_cast<char *>(host_scratch(ctx)) + kHostLzRingOffset);
}
// The ring as kernels address it.
LzRing *lz_ring_dev(rpb_ctx *ctx) {
  return reinterpret_cast<LzRing *>(static_cast<char *>(host_scratch_dev(ctx)) +
                                    kHostLzRingOffset);
}

// Waits for every ring copy still in flight (a previous call's last copy may target a slot
// this call is about to reuse, possibly from another stream).
int lz_ring_fence(rpb_ctx *ctx) {
  for (int q = 0; q < kLzRing; ++q) {
    if (!ctx->lz_live[q]) continue;
    RPB_HIP(ctx, hipEventSynchronize(ctx->lz_ev[q]));
    ctx->lz_live[q] = false;
  }
  return RPB_OK;
}

// Marks ring slot q with event q: the iteration's status-writing kernel (lanczos_eig or
// beta_eig, which store the status words into the slot) precedes it on the stream.
int lz_ring_post(rpb_ctx *ctx, int q, hipStream_t stream) {
  if (!ctx->lz_ev[q]) RPB_HIP(ctx, hipEventCreateWithFlags(&ctx->lz_ev[q], hipEventDisableTiming));
  RPB_HIP(ctx, hipEventRecord(ctx->lz_ev[q], stream));
  ctx->lz_live[q] = true;
  return RPB_OK;
}

// Blocks until the copy into ring slot q has landed.
int lz_ring_wait(rpb_ctx *ctx, int q) {
  RPB_HIP(ctx, hipEventSynchronize(ctx->lz_ev[q]));
  ctx->lz_live[q] = false;
  return RPB_OK;
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}



__global__ void scale_by_inverse(int64_t m, const double *__restrict__ x,
                                 const double *__restrict__ d, double *__restrict__ y,
                                 const LzState *__restrict__ st) {
  if (st && st->reason != 0) return;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double s = d[0];
  y[i] = s > 0.0 ? x[i] / s : 0.0;
}

// scale_by_inverse for v_{k+1} = u / beta_k that also writes it into the next product's
// packed sources, as that product's own packing would: src[c n + s] = Real(H_s y[3 s + c]).
template <typename Real>
__global__ void scale_by_inverse_packed(int64_t m, const double *__restrict__ x,
                                        const double *__restrict__ d, double *__restrict__ y,
                                        const LzState *__restrict__ st,
                                        const double *__restrict__ hw, Real *__restrict__ src) {
  if (st->reason != 0) return;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double s = d[0];
  const double v = s > 0.0 ? x[i] / s : 0.0;
  y[i] = v;
  const int64_t n = m / 3, sp = i / 3;
  src[(i - 3 * sp) * n + sp] = Real(hw[sp] * v);
}





// out = V y (first nvec rows of V)
__global__ void basis_combine(int64_t m, int nvec, const double *__restrict__ V,
                              const double *__restrict__ y, double *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double acc = 0.0;
  for (int k = 0; k < nvec; ++k) acc += y[k] * V[int64_t(k) * m + i];
  out[i] = acc;
}

// Eigendecomposition of T_{m-1} kept from one iteration to the next (the eigensolve of T_m
// updates it): eigenvalues in increasing order and the eigenvector matrix, row-major.
struct LzEig {
  double lam[kMaxKrylov];
  double Q[kMaxKrylov * kMaxKrylov];   // Q[col * kMaxKrylov + row] (column-major)
};

// 1/x: the hardware estimate refined by two Newton steps r <- r + r (1 - x r) (the error is
// squared by each; the result is within an ulp or two of the rounded quotient), about half the
// instructions of an IEEE division.  x finite and nonzero.
__device__ __forceinline__ double rcp_f64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

constexpr int kMaxRootIter = 64;   // secular-equation iterations per root before giving up

// The p + 1 roots of the secular equation of an arrowhead matrix with diagonal d (p distinct
// values, increasing), border z (no zero; z2 = z^2) and corner a:
//   f(mu) = a - mu - sum_j z_j^2 / (d_j - mu),
// decreasing between consecutive poles, so that root i lies in (d_{i-1}, d_i) (d_{-1} = -inf,
// d_p = +inf; the outer roots lie within |z| of d or a).  Root i is kept as mu = d_K + tau about
// its nearer pole K (the sign of f at the midpoint of the interval decides), with d_j - mu
// formed as (d_j - d_K) - tau, so that it keeps full relative accuracy in its distance to the
// pole.  Each step solves the model c + b tau + z_K^2 / tau = 0 (the pole K exact, the other
// terms linearised at the current tau: a quadratic with one root on each side of 0, the one on
// the side of the root is taken), safeguarded by bisection of the bracket; a root stops when
// |f| is within the rounding error of its terms, or when a step no longer moves it.
// Lane i of every wavefront follows root i; wavefront w sums the terms j = w, w + W, ... and
// the W partial sums are added in wavefront order through LDS, so every wavefront holds the
// same totals and takes the same steps.  Every thread of the workgroup calls this (W <=
// kThreads / 64); wavefront 0 writes K, tau, d_K and a failure flag (no stop within
// kMaxRootIter steps) for each root (K = -1, tau = 0 when p = 0: the root is a itself).
__device__ void secular_roots(int p, const double *__restrict__ d, const double *__restrict__ z2,
                              double a, int *K_out, double *tau_out, double *dK_out,
                              int *fail_out) {
  constexpr int kMaxW = kThreads / 64;
  __shared__ double part[2][kMaxW][4][64];
  __shared__ int more_s[2][kMaxW];
  const int w = int(threadIdx.x) / 64, i = int(threadIdx.x) & 63;
  // the terms are split over the wavefronts only when there are enough of them to pay for
  // the exchange (one barrier per step); otherwise the first wavefront takes them all
  const int W = p >= 16 ? int(blockDim.x) / 64 : 1;
  if (w >= W) return;   // wavefront-uniform; the caller's next barrier joins them again
  const bool act = p > 0 && i <= p;
  int buf = 0;
  // sums over all terms of w_j, |w_j|, and, without j = K, of w_j and w_j / (d_j - mu), with
  // w_j = z_j^2 / ((d_j - x0) - x1); with W > 1 also whether any wavefront reports `need`
  auto sums = [&](double x0, double x1, int K, bool need, double (&tot)[4]) -> bool {
    const bool any = __ballot(need) != 0ull;
    if (W == 1 && !any) return false;   // alone, the wavefront stops before summing again
    double f = 0.0, mag = 0.0, R = 0.0, Rp = 0.0;
    auto term = [&](int j, double inv) {
      const double t = z2[j] * inv;
      f += t;
      mag += fabs(t);
      if (j != K) {
        R += t;
        Rp += t * inv;
      }
    };
    if (act) {
      // four reciprocals in flight at a time; the sums still run in increasing j
      int j = w;
      for (; j + 3 * W < p; j += 4 * W) {
        double inv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) inv[r] = rcp_f64((d[j + r * W] - x0) - x1);
#pragma unroll
        for (int r = 0; r < 4; ++r) term(j + r * W, inv[r]);
      }
      for (; j < p; j += W) term(j, rcp_f64((d[j] - x0) - x1));
    }
    if (W == 1) {
      tot[0] = f;
      tot[1] = mag;
      tot[2] = R;
      tot[3] = Rp;
      return any;
    }
    part[buf][w][0][i] = f;
    part[buf][w][1][i] = mag;
    part[buf][w][2][i] = R;
    part[buf][w][3][i] = Rp;
    if (i == 0) more_s[buf][w] = any ? 1 : 0;
    __syncthreads();
    bool more = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double v = part[buf][0][q][i];
      for (int u = 1; u < W; ++u) v += part[buf][u][q][i];
      tot[q] = v;
    }
    for (int u = 0; u < W; ++u) more = more || more_s[buf][u] != 0;
    buf ^= 1;   // the next exchange uses the other buffer, so no second barrier is needed
    return more;
  };
  double zn2 = 0.0;
#pragma unroll 4
  for (int j = 0; j < p; ++j) zn2 += z2[j];
  const double znorm = sqrt(zn2);
  // bracket and pole of every root, and the first evaluation: an interior root at the midpoint
  // of its two poles (every term: the sign of f there picks the pole), an outer root half way
  // into its bracket about its only pole
  int K = 0;
  double lo = 0.0, hi = 0.0, x0 = 0.0, x1 = 0.0;
  if (act) {
    if (i == 0) {
      K = 0;
      lo = fmin(d[0], a) - znorm - d[0];
      x0 = d[0];
      x1 = 0.5 * lo;
    } else if (i == p) {
      K = p - 1;
      hi = fmax(d[p - 1], a) + znorm - d[p - 1];
      x0 = d[p - 1];
      x1 = 0.5 * hi;
    } else {
      K = -1;
      x0 = 0.5 * (d[i - 1] + d[i]);
    }
  }
  double tot[4];
  sums(x0, x1, K, true, tot);
  double tau = x1;
  if (act && i > 0 && i < p) {
    const double mid = x0;
    if ((a - mid) - tot[0] > 0.0) {   // the root lies above the midpoint: pole d_i
      K = i;
      lo = mid - d[i];
      tau = lo;
    } else {
      K = i - 1;
      hi = mid - d[i - 1];
      tau = hi;
    }
    // the sums without pole K, from those over every term
    const double inv = 1.0 / (d[K] - mid), t = z2[K] * inv;
    tot[2] -= t;
    tot[3] -= t * inv;
  }
  const double dK = act ? d[K] : 0.0, a0 = a - dK, zK2 = act ? z2[K] : 0.0;
  const bool above = K == i - 1;   // the root lies above its pole (tau > 0)
  bool done = !act, ok = !act;
  // every wavefront of the exchange sees the same `more`, so all take the same number of steps
  for (int it = 0; it == 0 || sums(dK, tau, K, !done, tot); ++it) {
    if (done) continue;
    const double f = (a0 - tau) - tot[0];
    const double mag = (fabs(a0) + fabs(tau)) + tot[1];
    if (fabs(f) <= 4.0 * DBL_EPSILON * mag) {
      done = ok = true;
      continue;
    }
    if (f > 0.0)
      lo = tau;
    else
      hi = tau;
    const double b = -1.0 - tot[3];           // slope of the linearised part
    const double c = (a0 - tau - tot[2]) - b * tau;
    const double disc = sqrt(c * c - 4.0 * b * zK2);
    // the quadratic's root on the side of the pole, in the form without cancellation
    const bool neg = c <= 0.0;
    const double num = above ? (neg ? 2.0 * zK2 : c + disc) : (neg ? disc - c : 2.0 * zK2);
    const double den = above ? (neg ? disc - c : -2.0 * b) : (neg ? 2.0 * b : -c - disc);
    double t = num * rcp_f64(den);
    if (!(t >= lo && t <= hi)) t = 0.5 * (lo + hi);
    if (fabs(t - tau) <= 2.0 * DBL_EPSILON * fabs(t)) done = ok = true;
    tau = t;
    if (it + 1 >= kMaxRootIter) done = true;
  }
  if (w == 0 && i <= p) {
    K_out[i] = act ? K : -1;
    tau_out[i] = act ? tau : 0.0;
    dK_out[i] = act ? dK : 0.0;
    fail_out[i] = ok ? 0 : 1;
  }
}

// Eigendecomposition of T_m from that of T_{m-1} (in eig, replaced by T_m's).  In the basis of
// T_{m-1}'s eigenvectors and e_m, T_m is an arrowhead matrix: diagonal lambda, border
// z = beta_{m-1} (last row of Q), corner alpha_m.  Its eigenproblem is solved as in the
// divide-and-conquer method (Cuppen 1981; Gu and Eisenstat 1995):
//   - deflation: a border entry below tol (8 eps |T|) leaves its lambda an eigenvalue; two
//     lambdas closer than tol / (c s) are rotated so that one border entry vanishes;
//   - the p + 1 roots of the secular equation of the rest, one lane each (secular_root);
//   - a border recomputed from the roots, z^_j^2 = prod_i |d_j - mu_i| / prod_{l != j}
//     |d_j - d_l| (the border for which the computed roots are exact), which keeps the
//     eigenvectors u_i = (z^_j / (d_j - mu_i), -1) / norm orthogonal to working accuracy;
//   - new eigenvectors [Q 0; 0 1] U and the eigenvalues sorted increasingly.
// Every thread of the workgroup calls this; the first wavefront (one lane per eigenvalue, m <=
// 64) does the scalar work and the workgroup forms the product.  Returns 1 (every thread)
// when a root iteration did not stop or an eigenvalue is not finite.
__device__ int eig_update(int m, const LzState *__restrict__ st, LzEig *__restrict__ eig) {
  // column-major (entry [row or component] fastest), so that the lanes of a wavefront, which
  // take consecutive rows, touch consecutive LDS words
  __shared__ double Qs[kMaxKrylov * kMaxKrylov];   // old Q (rows < m - 1), rotated: [col * 64 + row]
  __shared__ double U[kMaxKrylov * kMaxKrylov];    // eigenvectors of the arrowhead: [j * 64 + i]
  __shared__ double Qk[kMaxKrylov * kMaxKrylov];   // the kept columns of Qs, in order
  __shared__ double dd[kMaxKrylov], zz[kMaxKrylov], dn[kMaxKrylov], z2n[kMaxKrylov];
  __shared__ double zh[kMaxKrylov], tau_s[kMaxKrylov], dK_s[kMaxKrylov], val[kMaxKrylov];
  __shared__ double rot_c[kMaxKrylov], rot_s[kMaxKrylov];
  __shared__ int K_s[kMaxKrylov], nd_s[kMaxKrylov], df_s[kMaxKrylov], rank_s[kMaxKrylov];
  __shared__ int fail_s[kMaxKrylov];
  __shared__ int rot_p[kMaxKrylov], rot_j[kMaxKrylov];
  __shared__ int info[4];   // p, number of deflated, number of rotations, failure
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63;
  const bool w0 = tid < 64;
  if (m == 1) {
    if (tid == 0) {
      eig->lam[0] = st->alpha[0];
      eig->Q[0] = 1.0;
    }
    __syncthreads();
    return 0;
  }
  const int n1 = m - 1;
  const double alpha = st->alpha[m - 1], beta = st->beta[m - 2];
  for (int e = tid; e < n1 * n1; e += nthr) {
    const int c = e / n1, r = e - c * n1;
    Qs[c * 64 + r] = eig->Q[c * kMaxKrylov + r];
  }
  if (w0) {
    if (lane < n1) {
      dd[lane] = eig->lam[lane];
      zz[lane] = beta * eig->Q[lane * kMaxKrylov + (n1 - 1)];
    }
    // deflation tolerance from |T_m| <= max(|lambda|, |alpha|) + |beta|
    double amax = lane < n1 ? fabs(eig->lam[lane]) : 0.0;
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
    const double tol = 8.0 * DBL_EPSILON * (fmax(amax, fabs(alpha)) + fabs(beta));
    // the wavefront's LDS accesses complete in order: dd and zz are visible below
    const double zj = lane < n1 ? zz[lane] : 0.0;
    unsigned long long keep = __ballot(lane < n1 && fabs(zj) > tol);
    // a kept entry and the kept entry before it that would rotate into one (parallel test;
    // the rotations themselves are taken in order, below, only when some pair qualifies)
    bool close = false;
    if ((keep >> lane) & 1ull) {
      const unsigned long long below = keep & ((1ull << lane) - 1ull);
      if (below) {
        const int q = 63 - __builtin_clzll(below);
        const double zq = zz[q], r = sqrt(zq * zq + zj * zj);
        close = fabs((zj / r) * (zq / r) * (dd[lane] - dd[q])) <= tol;
      }
    }
    int nrot = 0;
    if (__ballot(close)) {
      // in order over the entries, every lane alike: a kept entry q followed by a kept j
      // whose rotation deflates q
      keep = 0;
      int prev = -1;
      for (int j = 0; j < n1; ++j) {
        const double zjj = zz[j];
        if (!(fabs(zjj) > tol)) continue;
        if (prev >= 0) {
          const double zp = zz[prev], r = sqrt(zp * zp + zjj * zjj);
          const double c = zjj / r, sn = zp / r;
          if (fabs(c * sn * (dd[j] - dd[prev])) <= tol) {
            const double dp = dd[prev], dj = dd[j];
            if (lane == 0) {
              dd[prev] = c * c * dp + sn * sn * dj;
              dd[j] = sn * sn * dp + c * c * dj;
              zz[prev] = 0.0;
              zz[j] = r;
              rot_p[nrot] = prev;
              rot_j[nrot] = j;
              rot_c[nrot] = c;
              rot_s[nrot] = sn;
            }
            ++nrot;
            keep &= ~(1ull << prev);
          }
        }
        keep |= 1ull << j;
        prev = j;
      }
    }
    const int p = __popcll(keep);
    const unsigned long long lower = (1ull << lane) - 1ull;
    if (lane < n1) {
      if ((keep >> lane) & 1ull) {
        const int q = __popcll(keep & lower);
        dn[q] = dd[lane];
        z2n[q] = zz[lane] * zz[lane];
        nd_s[q] = lane;
      } else {
        df_s[__popcll(~keep & lower)] = lane;
      }
    }
    if (lane == 0) {
      info[0] = p;
      info[1] = n1 - p;
      info[2] = nrot;
    }
  }
  __syncthreads();
  const int p = info[0], ndf = info[1], nrot = info[2];
  // the deflating rotations on the columns of the old Q, in order
  for (int q = 0; q < nrot; ++q) {
    const int a = rot_p[q], b = rot_j[q];
    const double c = rot_c[q], sn = rot_s[q];
    for (int r = tid; r < n1; r += nthr) {
      const double qa = Qs[a * 64 + r], qb = Qs[b * 64 + r];
      Qs[a * 64 + r] = c * qa - sn * qb;
      Qs[b * 64 + r] = sn * qa + c * qb;
    }
    __syncthreads();
  }
  // the kept columns side by side for the product below (read after the next barrier)
  for (int x = tid; x < p * n1; x += nthr) {
    const int jj = x / n1, r = x - jj * n1;
    Qk[jj * 64 + r] = Qs[nd_s[jj] * 64 + r];
  }
  // the roots (with p = 0 the arrowhead is alpha alone), by the whole workgroup
  secular_roots(p, dn, z2n, alpha, K_s, tau_s, dK_s, fail_s);
  if (w0) {
    int bad = 0;
    if (lane <= p) {
      bad = fail_s[lane];
      const int K = K_s[lane];
      val[lane] = K >= 0 ? dK_s[lane] + tau_s[lane] : alpha;
    } else if (lane < m) {
      val[lane] = dd[df_s[lane - p - 1]];
    }
    // the recomputed border: the numerator's roots paired with the denominator's poles
    if (lane < p) {
      const double dj = dn[lane];
      // each factor formed apart from the running product, so that only a multiply waits on it
      double prod = 1.0;
#pragma unroll 4
      for (int i = 0; i <= p; ++i) {
        const double num = fabs((dj - dK_s[i]) - tau_s[i]);
        prod *= (i < p && i != lane) ? num * rcp_f64(fabs(dj - dn[i])) : num;
      }
      zh[lane] = sqrt(prod);   // its sign: that of the border entry, which z2n does not keep
      const double zs = zz[nd_s[lane]];
      if (zs < 0.0) zh[lane] = -zh[lane];
    }
    // eigenvector lane of the arrowhead (entries 0..p-1 on the kept lambdas, p on e_m)
    if (lane <= p) {
      double nrm = 1.0;
      if (p > 0) {
        const int K = K_s[lane];
        const double dK = dn[K], tau = tau_s[lane];
#pragma unroll 4
        for (int j = 0; j < p; ++j) {
          const double x = zh[j] * rcp_f64((dn[j] - dK) - tau);
          U[j * 64 + lane] = x;
          nrm += x * x;
        }
      }
      const double inv = 1.0 / sqrt(nrm);
#pragma unroll 4
      for (int j = 0; j < p; ++j) U[j * 64 + lane] *= inv;
      U[p * 64 + lane] = -inv;
    }
    // rank of every eigenvalue (ties by index)
    if (lane < m) {
      const double v = val[lane];
      int r = 0;
#pragma unroll 8
      for (int e = 0; e < m; ++e) {
        const double ve = val[e];
        r += (ve < v || (ve == v && e < lane)) ? 1 : 0;
      }
      rank_s[lane] = r;
      eig->lam[r] = v;
      bad |= !isfinite(v);
    }
    bad = __ballot(bad) != 0ull;
    if (lane == 0) info[3] = bad;
  }
  __syncthreads();
  // new eigenvectors: column rank(e) of Q_m, rows 0..m-1
  for (int x = tid; x < m * m; x += nthr) {
    const int e = x / m, r = x - e * m;
    double v;
    if (e <= p) {
      if (r < n1) {
        // four running sums keep several LDS loads in flight
        double v4[4] = {0.0, 0.0, 0.0, 0.0};
        int j = 0;
        for (; j + 4 <= p; j += 4)
#pragma unroll
          for (int q = 0; q < 4; ++q) v4[q] += Qk[(j + q) * 64 + r] * U[(j + q) * 64 + e];
        for (; j < p; ++j) v4[0] += Qk[j * 64 + r] * U[j * 64 + e];
        v = (v4[0] + v4[1]) + (v4[2] + v4[3]);
      } else {
        v = U[p * 64 + e];
      }
    } else {
      v = r < n1 ? Qs[df_s[e - p - 1] * 64 + r] : 0.0;
    }
    eig->Q[rank_s[e] * kMaxKrylov + r] = v;
  }
  __syncthreads();
  return info[3];
}

// Eigendecomposition of T_m (eig_update), then y_m = |w| Q L^{1/2} Q^T e_1, eps_m and the stop
// test.  Every thread of the workgroup calls this; the first wavefront forms y_m and the status.
__device__ void tridiag_body(int m, double tol, LzState *__restrict__ st, LzEig *__restrict__ eig) {
  __shared__ double Rz[kMaxKrylov];   // sqrt(lambda_k) q_k[0]
  const int failed = eig_update(m, st, eig);
  const int lane = threadIdx.x;
  if (lane >= 64) return;
  const double lmin = eig->lam[0], lmax = eig->lam[m - 1];
  double amax = lane < m ? fabs(st->alpha[lane]) : 0.0;
  for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
  // y_m = |w| Q L^{1/2} Q^T e_1: lane k forms sqrt(lambda_k) q_k[0], then lane r sums row r
  if (lane < m) Rz[lane] = sqrt(fmax(eig->lam[lane], 0.0)) * eig->Q[lane * kMaxKrylov];
  const double wn = st->wnorm;
  double yr = 0.0;
  if (lane < m) {
#pragma unroll 4
    for (int k = 0; k < m; ++k) yr += Rz[k] * eig->Q[k * kMaxKrylov + lane];
    yr *= wn;
  }
  // eps_m in the orthonormal Krylov basis
  const double yp = (lane < m - 1) ? st->yprev[lane] : 0.0;
  const double diff = (lane < m) ? (yr - yp) : 0.0;
  double num = diff * diff, den = yp * yp;
  for (int off = 32; off > 0; off >>= 1) {
    num += __shfl_xor(num, off, 64);
    den += __shfl_xor(den, off, 64);
  }
  if (lane < m) {
    st->y[lane] = yr;
    st->yprev[lane] = yr;
  }
  if (lane == 0) {
    const double eps = m >= 2 ? sqrt(num / den) : 0.0;
    int reason = 0;
    if (failed)
      reason = 4;
    else if (lmin < -1e-12 * fmax(lmax, 0.0))
      reason = 3;
    else if (m >= 2 && eps < tol)
      reason = 1;
    else if (st->beta[m - 1] <= 1e-14 * amax)
      reason = 2;
    st->eps = eps;
    st->m = m;
    st->reason = reason;
  }
}

// Status words of the iteration into the host's ring slot (pinned host memory, written by the
// kernel so that no copy needs enqueuing), by one thread after the state is final.
__device__ __forceinline__ void post_status(const LzState *__restrict__ st, LzRingSlot *slot) {
  slot->eps = st->eps;
  slot->m = st->m;
  slot->reason = st->reason;
  __threadfence_system();
}

__global__ void lz_reset(LzState *st) {
  const int t = threadIdx.x;
  if (t < kMaxKrylov) {
    st->alpha[t] = 0.0;
    st->beta[t] = 0.0;
    st->y[t] = 0.0;
    st->yprev[t] = 0.0;
    st->h[t] = 0.0;
  }
  if (t == 0) {
    st->wnorm = 0.0;
    st->halt = 0;
    st->eps = 0.0;
    st->m = 0;
    st->reason = 0;
  }
}

// ---- one Lanczos iteration of a single system in six kernels (segments > kFusedSegment) ----
//
// Sums in two stages, kRedBlocks workgroup partials and their sum in a fixed order by one
// workgroup (a last-arriving workgroup could take the second stage, but its device-scope
// release fence writes back its XCD's L2 and cost more than the launch it saved).  The
// three-term recurrence is applied where its result is read; alpha's second stage is taken by
// every workgroup of the re-orthogonalisation dots (the same sum in each), and the second
// stage of |u| shares its workgroup with the eigensolve.  The arithmetic and its order are
// those of one kernel per step.

__global__ __launch_bounds__(kThreads) void dot_partial(int64_t m, const double *__restrict__ a,
                                                        const double *__restrict__ b,
                                                        double *__restrict__ part) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < m;
       i += int64_t(gridDim.x) * kThreads)
    acc += a[i] * b[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out = sum(part) (mode 0) or sqrt(sum(part)) (mode 1)
__global__ __launch_bounds__(kThreads) void dot_finish(const double *__restrict__ part, int np,
                                                       double *__restrict__ out, int mode) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += kThreads) acc += part[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[0] = mode == 1 ? sqrt(s) : s;
}

// part[j * gridDim.x + b] = partial of V_j . (u - alpha_k v_k - beta_{k-1} v_{k-1}) over
// workgroup b's share (grid y: j < k); u is not modified.  alpha_k is the sum of the np
// partials of v_k . u in apart, which every workgroup forms as dot_finish would (the same
// value in each), and the first workgroup stores (alpha_out).
__global__ __launch_bounds__(kThreads) void reorth_dots_3t(
    int64_t m, const double *__restrict__ V, const double *__restrict__ u,
    const double *__restrict__ vk, const double *__restrict__ vprev,
    const double *__restrict__ apart, int np, double *__restrict__ alpha_out,
    const double *__restrict__ beta, double *__restrict__ part) {
  __shared__ double sh[kThreads];
  double a0 = 0.0;
  for (int i = threadIdx.x; i < np; i += kThreads) a0 += apart[i];
  const double al = block_sum(a0, sh);
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) alpha_out[0] = al;
  const int j = blockIdx.y;
  const double *vj = V + int64_t(j) * m;
  const double be = vprev ? beta[0] : 0.0;
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < m;
       i += int64_t(gridDim.x) * kThreads) {
    double x = u[i] - al * vk[i];
    if (vprev) x -= be * vprev[i];
    acc += vj[i] * x;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[int64_t(j) * gridDim.x + blockIdx.x] = s;
}

// h[j] = sum of the np partials of V_j . u; one workgroup per basis vector j
__global__ __launch_bounds__(kThreads) void reorth_finish(int np, const double *__restrict__ part,
                                                          double *__restrict__ h) {
  __shared__ double sh[kThreads];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += kThreads) acc += part[int64_t(j) * np + i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) h[j] = s;
}

// u <- u - alpha_k v_k - beta_{k-1} v_{k-1} - sum_j h_j V_j, and the workgroup partials of |u|^2
__global__ __launch_bounds__(kThreads) void reorth_update_sq(
    int64_t m, int k, const double *__restrict__ V, double *__restrict__ u,
    const double *__restrict__ vk, const double *__restrict__ vprev,
    const LzState *__restrict__ st, double *__restrict__ part) {
  __shared__ double sh[kThreads];
  const double al = st->alpha[k - 1], be = vprev ? st->beta[k - 2] : 0.0;
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < m;
       i += int64_t(gridDim.x) * kThreads) {
    double x = u[i] - al * vk[i];
    if (vprev) x -= be * vprev[i];
    double proj = 0.0;
    for (int j = 0; j < k; ++j) proj += st->h[j] * V[int64_t(j) * m + i];
    x -= proj;
    u[i] = x;
    acc += x * x;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// beta_k = sqrt(sum of the np partials), then the eigensolve of T_k with its stop test (unless
// the process has stopped) and the status words into the host's ring slot.
__global__ __launch_bounds__(kThreads) void beta_eig(int np, const double *__restrict__ part,
                                                     int k, double tol, LzState *__restrict__ st,
                                                     LzEig *__restrict__ eig, LzRingSlot *slot) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += kThreads) acc += part[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) st->beta[k - 1] = sqrt(s);
  __syncthreads();
  // every thread reads the same reason: only tridiag_body writes it, after its barriers
  if (st->reason == 0) tridiag_body(k, tol, st, eig);
  if (threadIdx.x == 0) post_status(st, slot);
}

// Longest segment (3 n values of one system) that one workgroup takes through a whole Lanczos
// iteration (lanczos_step_body); longer segments use the multi-workgroup reductions.  One
// workgroup keeps too few loads in flight for much longer segments: with 8,192 spheres per
// system the 64-system batched step was 18 % slower than with the separate kernels.
constexpr int64_t kFusedSegment = 3 * 512;

// The vector work and the eigensolve of Lanczos iteration k for the segment [e0, e1) of the
// vectors, by one workgroup, after the product u = M v_k: alpha_k = v_k . u; u -= alpha_k v_k +
// beta_{k-1} v_{k-1}; the full re-orthogonalisation u -= V_k (V_k^T u); beta_k = |u|; the
// eigensolve of T_k with its stop test (tridiag_body); and, unless the process stopped,
// v_{k+1} = u / beta_k (when write_next).  The steps and their order are those of the separate
// kernels; the sums are taken over the workgroup instead of in two stages, so small systems
// need one launch per iteration instead of about ten.
// Sums over the workgroup of NV values per thread, each returned to every thread: a butterfly
// over the wavefront's 64 lanes, then the kThreads/64 wavefront sums added in a fixed order.
template <int NV>
__device__ __forceinline__ void group_sums(double (&v)[NV], double *sh) {
  constexpr int W = kThreads / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q)
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[q * W + wave] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double r = sh[q * W];
    for (int w = 1; w < W; ++w) r += sh[q * W + w];
    v[q] = r;
  }
  __syncthreads();
}

// The vector work (alpha_k, the recurrence, the re-orthogonalisation, beta_k; alpha, beta and
// the projections h stored in st), leaving the unnormalised u; returns beta_k to every thread.
// The segment has at most kEpt values per thread (kFusedSegment in all), so each thread keeps
// its values of u, v_k and v_{k-1} in registers, and each pass over the basis issues all its
// loads at once; the sums and their order are those of one value at a time.
constexpr int kMaxEpt = int(kFusedSegment / kThreads);
static_assert(kFusedSegment % kThreads == 0, "whole values per thread");
template <int kEpt>
__device__ __forceinline__ double lanczos_vec_values(LzState *__restrict__ st,
                                                     const double *__restrict__ V,
                                                     double *__restrict__ u, int64_t m3,
                                                     int64_t e0, int64_t e1, int k) {
  constexpr int W = kThreads / 64;
  __shared__ double sh[8 * W];
  __shared__ double hsh[kMaxKrylov * W];   // wavefront sums of h_j: [j * W + wave]
  __shared__ double hs[kMaxKrylov];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const double *vk = V + int64_t(k - 1) * m3;
  const double *vp = k > 1 ? V + int64_t(k - 2) * m3 : nullptr;
  // this thread's values: element e0 + t + r kThreads, r < kEpt (clamped loads past e1)
  bool in[kEpt];
  int64_t ix[kEpt];
  double uu[kEpt], xv[kEpt];
#pragma unroll
  for (int r = 0; r < kEpt; ++r) {
    const int64_t i = e0 + t + int64_t(r) * kThreads;
    in[r] = i < e1;
    ix[r] = in[r] ? i : e0;
  }
#pragma unroll
  for (int r = 0; r < kEpt; ++r) uu[r] = u[ix[r]];
#pragma unroll
  for (int r = 0; r < kEpt; ++r) xv[r] = vk[ix[r]];
  double acc[1] = {0.0};
#pragma unroll
  for (int r = 0; r < kEpt; ++r)
    if (in[r]) acc[0] += xv[r] * uu[r];
  group_sums(acc, sh);
  const double alpha = acc[0];
  const double bprev = k > 1 ? st->beta[k - 2] : 0.0;
  double pv[kEpt];
#pragma unroll
  for (int r = 0; r < kEpt; ++r) pv[r] = vp ? vp[ix[r]] : 0.0;
#pragma unroll
  for (int r = 0; r < kEpt; ++r) {
    double x = uu[r] - alpha * xv[r];
    if (vp) x -= bprev * pv[r];
    uu[r] = x;
  }
  // h_j = V_j . u for j < k, eight basis vectors per pass (past the last vector the loads
  // reread it and add nothing); each wavefront's sums go to LDS, added over the wavefronts
  // in a fixed order after the last pass
  for (int j0 = 0; j0 < k; j0 += 8) {
    const int nj = min(8, k - j0);
    double vq[8][kEpt];
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int r = 0; r < kEpt; ++r) vq[q][r] = V[int64_t(min(j0 + q, k - 1)) * m3 + ix[r]];
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < kEpt; ++r)
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (in[r] && q < nj) a[q] += vq[q][r] * uu[r];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      for (int off = 32; off > 0; off >>= 1) a[q] += __shfl_xor(a[q], off, 64);
    if (lane == 0)
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < nj) hsh[(j0 + q) * W + wave] = a[q];
  }
  __syncthreads();
  if (t < k) {
    double r = hsh[t * W];
    for (int w = 1; w < W; ++w) r += hsh[t * W + w];
    hs[t] = r;
  }
  __syncthreads();
  // u -= V_k h: per value the terms in increasing j, eight basis vectors' loads at a time
  double proj[kEpt];
#pragma unroll
  for (int r = 0; r < kEpt; ++r) proj[r] = 0.0;
  for (int j0 = 0; j0 < k; j0 += 8) {
    const int nj = min(8, k - j0);
    double vq[8][kEpt];
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int r = 0; r < kEpt; ++r) vq[q][r] = V[int64_t(min(j0 + q, k - 1)) * m3 + ix[r]];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double hj = q < nj ? hs[j0 + q] : 0.0;
#pragma unroll
      for (int r = 0; r < kEpt; ++r)
        if (q < nj) proj[r] += hj * vq[q][r];
    }
  }
  acc[0] = 0.0;
#pragma unroll
  for (int r = 0; r < kEpt; ++r) {
    uu[r] -= proj[r];
    if (in[r]) {
      u[ix[r]] = uu[r];
      acc[0] += uu[r] * uu[r];
    }
  }
  group_sums(acc, sh);
  const double beta = sqrt(acc[0]);
  if (t == 0) {
    st->alpha[k - 1] = alpha;
    st->beta[k - 1] = beta;
  }
  if (t < k) st->h[t] = hs[t];
  return beta;
}

// lanczos_vec_values with as many values per thread as the segment needs (workgroup-uniform)
__device__ __forceinline__ double lanczos_vec_body(LzState *__restrict__ st,
                                                   const double *__restrict__ V,
                                                   double *__restrict__ u, int64_t m3,
                                                   int64_t e0, int64_t e1, int k) {
  static_assert(kMaxEpt == 6, "one case per count of values per thread");
  switch (int((e1 - e0 + kThreads - 1) / kThreads)) {
    case 0:
    case 1: return lanczos_vec_values<1>(st, V, u, m3, e0, e1, k);
    case 2: return lanczos_vec_values<2>(st, V, u, m3, e0, e1, k);
    case 3: return lanczos_vec_values<3>(st, V, u, m3, e0, e1, k);
    case 4: return lanczos_vec_values<4>(st, V, u, m3, e0, e1, k);
    case 5: return lanczos_vec_values<5>(st, V, u, m3, e0, e1, k);
    default: return lanczos_vec_values<6>(st, V, u, m3, e0, e1, k);
  }
}

// v_{k+1} = u / beta_k on [e0, e1) (0 when beta_k = 0)
__device__ __forceinline__ void lanczos_write_next(double *__restrict__ V,
                                                   const double *__restrict__ u, int64_t m3,
                                                   int64_t e0, int64_t e1, int k, double beta) {
  double *next = V + int64_t(k) * m3;
  for (int64_t i = e0 + threadIdx.x; i < e1; i += kThreads)
    next[i] = beta > 0.0 ? u[i] / beta : 0.0;
}

// The vector work and the eigensolve of Lanczos iteration k for the segment [e0, e1) of the
// vectors, by one workgroup: lanczos_vec_body, the eigensolve of T_k with its stop test
// (tridiag_body) and, unless the process stopped, v_{k+1} (when write_next).
__device__ void lanczos_step_body(LzState *__restrict__ st, LzEig *__restrict__ eig,
                                  double *__restrict__ V, double *__restrict__ u, int64_t m3,
                                  int64_t e0, int64_t e1, int k, double tol, bool write_next) {
  const double beta = lanczos_vec_body(st, V, u, m3, e0, e1, k);
  __syncthreads();
  tridiag_body(k, tol, st, eig);
  __syncthreads();
  if (write_next && st->reason == 0) lanczos_write_next(V, u, m3, e0, e1, k, beta);
}

// Single system, the whole vector (3 n <= kFusedSegment): the vector work of iteration k and
// v_{k+1}, with the eigensolve and stop test left to lanczos_eig on a second stream, which
// runs beside the next product.  Until that stream reports a stop the recurrence runs on (the
// iterations past the stop are never used); once the workgroup sees reason != 0 it only sets
// st->halt, on which the products of later iterations return at once.  (reason is written by
// the other stream meanwhile: one thread reads it and the workgroup follows that read.)
// With src (nullable), v_{k+1} also goes into the next product's packed sources, as that
// product's own packing would write them: src[c n + s] = Real(H_s v_{k+1}[3 s + c]) (hw: H).
template <typename Real>
__global__ __launch_bounds__(kThreads) void lanczos_vec(LzState *__restrict__ st,
                                                        double *__restrict__ V,
                                                        double *__restrict__ u, int64_t m3, int k,
                                                        int write_next,
                                                        const double *__restrict__ hw,
                                                        Real *__restrict__ src) {
  __shared__ int stop_s;
  if (threadIdx.x == 0) {
    stop_s = __hip_atomic_load(&st->reason, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    if (stop_s) st->halt = 1;
  }
  __syncthreads();
  if (stop_s) return;
  const double beta = lanczos_vec_body(st, V, u, m3, 0, m3, k);
  if (!write_next) return;
  double *next = V + int64_t(k) * m3;
  const int64_t n = m3 / 3;
  for (int64_t i = threadIdx.x; i < m3; i += kThreads) {
    const double x = beta > 0.0 ? u[i] / beta : 0.0;
    next[i] = x;
    if (src) {
      const int64_t s = i / 3;
      src[(i - 3 * s) * n + s] = Real(hw[s] * x);
    }
  }
}

// The eigensolve of T_k and the stop test (skipped once the process has stopped: y, eps and
// reason stay), then the status into the host's ring slot.  Only these kernels write reason,
// one after another on their stream, so every thread reads the same value.
__global__ __launch_bounds__(kThreads) void lanczos_eig(LzState *__restrict__ st,
                                                        LzEig *__restrict__ eig, int k,
                                                        double tol, LzRingSlot *slot) {
  if (st->reason == 0) tridiag_body(k, tol, st, eig);
  if (threadIdx.x == 0) post_status(st, slot);
}

// ---- batched Lanczos: one Krylov process per system, segments of the concatenated vectors ----
//
// System s owns elements [3 offs[s], 3 offs[s+1]) of every 3n vector and its own LzState.
// done[s] != 0 freezes a system: every kernel skips it, so a system stops changing once its
// own tolerance or breakdown test is met, whatever the others do.

constexpr int kSegBlocks = 16;      // partial sums per system segment

struct SegView {
  const int64_t *offs;    // nsys + 1 (device)
  const int *sys_of;      // sphere -> system (device)
  LzState *st;            // nsys states
  int *done;              // nsys flags
  LzEig *eig;             // nsys eigendecompositions
};

// part[s * kSegBlocks + b] = partial dot of a and b over system s
__global__ __launch_bounds__(kThreads) void seg_dot_partial(SegView v, const double *__restrict__ a,
                                                            const double *__restrict__ b,
                                                            double *__restrict__ part) {
  __shared__ double sh[kThreads];
  const int s = blockIdx.y;
  if (v.done[s]) return;
  const int64_t e0 = 3 * v.offs[s], e1 = 3 * v.offs[s + 1];
  double acc = 0.0;
  for (int64_t i = e0 + int64_t(blockIdx.x) * kThreads + threadIdx.x; i < e1;
       i += int64_t(kSegBlocks) * kThreads)
    acc += a[i] * b[i];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) part[int64_t(s) * kSegBlocks + blockIdx.x] = r;
}

// st[s].<field at double offset `field`> = sum (mode 0) or sqrt(sum) (mode 1)
__global__ __launch_bounds__(64) void seg_dot_finish(SegView v, const double *__restrict__ part,
                                                     int field, int mode) {
  const int s = blockIdx.x;
  if (v.done[s] || threadIdx.x != 0) return;
  double acc = 0.0;
  for (int b = 0; b < kSegBlocks; ++b) acc += part[int64_t(s) * kSegBlocks + b];
  reinterpret_cast<double *>(v.st + s)[field] = mode == 1 ? sqrt(acc) : acc;
}

// y = x / st[s].<field> on every live system (zero when the divisor is not positive)
__global__ void seg_scale_by_inverse(SegView v, int64_t m, const double *__restrict__ x, int field,
                                     double *__restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int s = v.sys_of[i / 3];
  if (v.done[s]) return;
  const double d = reinterpret_cast<const double *>(v.st + s)[field];
  y[i] = d > 0.0 ? x[i] / d : 0.0;
}

// part[(s * nvec + j) * kSegBlocks + b] = partial dot of V_j and u - alpha_k v_k -
// beta_{k-1} v_{k-1} over system s (the three-term recurrence applied where it is read; u is
// not modified), nvec = k
__global__ __launch_bounds__(kThreads) void seg_reorth_dots_3t(
    SegView v, int64_t m, int nvec, const double *__restrict__ V, const double *__restrict__ u,
    const double *__restrict__ vk, const double *__restrict__ vprev, double *__restrict__ part) {
  __shared__ double sh[kThreads];
  const int s = blockIdx.z, j = blockIdx.y;
  if (v.done[s]) return;
  const int64_t e0 = 3 * v.offs[s], e1 = 3 * v.offs[s + 1];
  const double *vj = V + int64_t(j) * m;
  const double al = v.st[s].alpha[nvec - 1], be = vprev ? v.st[s].beta[nvec - 2] : 0.0;
  double acc = 0.0;
  for (int64_t i = e0 + int64_t(blockIdx.x) * kThreads + threadIdx.x; i < e1;
       i += int64_t(kSegBlocks) * kThreads) {
    double x = u[i] - al * vk[i];
    if (vprev) x -= be * vprev[i];
    acc += vj[i] * x;
  }
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) part[(int64_t(s) * nvec + j) * kSegBlocks + blockIdx.x] = r;
}

__global__ __launch_bounds__(64) void seg_reorth_finish(SegView v, int nvec,
                                                        const double *__restrict__ part) {
  const int s = blockIdx.x;
  if (v.done[s]) return;
  for (int j = threadIdx.x; j < nvec; j += blockDim.x) {
    double acc = 0.0;
    for (int b = 0; b < kSegBlocks; ++b) acc += part[(int64_t(s) * nvec + j) * kSegBlocks + b];
    v.st[s].h[j] = acc;
  }
}

// u <- u - alpha_k v_k - beta_{k-1} v_{k-1} - sum_j h_j V_j on every live system, and
// part[s * kSegBlocks + b] = the partial of |u|^2 over system s
__global__ __launch_bounds__(kThreads) void seg_reorth_update_sq(
    SegView v, int64_t m, int k, const double *__restrict__ V, double *__restrict__ u,
    const double *__restrict__ vk, const double *__restrict__ vprev, double *__restrict__ part) {
  __shared__ double sh[kThreads];
  const int s = blockIdx.y;
  if (v.done[s]) return;
  const int64_t e0 = 3 * v.offs[s], e1 = 3 * v.offs[s + 1];
  const LzState &st = v.st[s];
  const double al = st.alpha[k - 1], be = vprev ? st.beta[k - 2] : 0.0;
  double acc = 0.0;
  for (int64_t i = e0 + int64_t(blockIdx.x) * kThreads + threadIdx.x; i < e1;
       i += int64_t(kSegBlocks) * kThreads) {
    double x = u[i] - al * vk[i];
    if (vprev) x -= be * vprev[i];
    double proj = 0.0;
    for (int j = 0; j < k; ++j) proj += st.h[j] * V[int64_t(j) * m + i];
    x -= proj;
    u[i] = x;
    acc += x * x;
  }
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) part[int64_t(s) * kSegBlocks + blockIdx.x] = r;
}

// beta_k = sqrt(sum of the system's kSegBlocks partials, in order), then the eigensolve of T_k
// with its stop test; a stopped system is frozen.
__global__ __launch_bounds__(64) void seg_beta_eig(SegView v, int m, double tol,
                                                   const double *__restrict__ part) {
  const int s = blockIdx.x;
  if (v.done[s]) return;
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int b = 0; b < kSegBlocks; ++b) acc += part[int64_t(s) * kSegBlocks + b];
    v.st[s].beta[m - 1] = sqrt(acc);
  }
  __syncthreads();
  tridiag_body(m, tol, v.st + s, v.eig + s);
  if (threadIdx.x == 0 && v.st[s].reason != 0) v.done[s] = 1;
}

// The eigensolve of T_1, T_2, ..., T_m in turn (as a Krylov process meets them), row k - 1 of
// ys (m doubles) receiving y_k = |w| T_k^{1/2} e_1 (entries k..m-1 zero); fail[0] = 1 when an
// eigensolve fails.  The stop tests are evaluated but do not stop the sequence.
__global__ __launch_bounds__(64) void tridiag_sequence(int m, LzState *__restrict__ st,
                                                       LzEig *__restrict__ eig,
                                                       double *__restrict__ ys,
                                                       int *__restrict__ fail) {
  const int t = threadIdx.x;
  if (t == 0) fail[0] = 0;
  for (int k = 1; k <= m; ++k) {
    tridiag_body(k, 0.0, st, eig);
    __syncthreads();
    if (t < m) ys[int64_t(k - 1) * m + t] = t < k ? st->y[t] : 0.0;
    if (t == 0 && st->reason == 4) fail[0] = 1;
    __syncthreads();
  }
}

// lanczos_step_body for every live system, one workgroup each (segments <= kFusedSegment).
__global__ __launch_bounds__(kThreads) void seg_lanczos_step(SegView v, double *__restrict__ V,
                                                             double *__restrict__ u, int64_t m3,
                                                             int k, double tol, int write_next) {
  const int s = blockIdx.x;
  if (v.done[s]) return;
  LzState *st = v.st + s;
  lanczos_step_body(st, v.eig + s, V, u, m3, 3 * v.offs[s], 3 * v.offs[s + 1], k, tol,
                    write_next != 0);
  if (threadIdx.x == 0 && st->reason != 0) v.done[s] = 1;
}

// out = V_m y_m per system (m = the system's own iteration count)
__global__ void seg_basis_combine(SegView v, int64_t m, const double *__restrict__ V,
                                  double *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const LzState &st = v.st[v.sys_of[i / 3]];
  double acc = 0.0;
  for (int j = 0; j < st.m; ++j) acc += st.y[j] * V[int64_t(j) * m + i];
  out[i] = acc;
}

__global__ void lz_reset_batched(SegView v, int nsys) {
  const int s = blockIdx.x;
  if (s >= nsys) return;
  LzState *st = v.st + s;
  const int t = threadIdx.x;
  if (t < kMaxKrylov) {
    st->alpha[t] = 0.0;
    st->beta[t] = 0.0;
    st->y[t] = 0.0;
    st->yprev[t] = 0.0;
    st->h[t] = 0.0;
  }
  if (t == 0) {
    st->wnorm = 0.0;
    st->eps = 0.0;
    st->m = 0;
    st->reason = 0;
    v.done[s] = 0;
    if (s == 0) v.done[nsys] = 0;
  }
}

// done[nsys] = 1 once every system is done: later launches of the persistent product kernel
// return at once instead of walking their work list.
__global__ __launch_bounds__(256) void seg_all_done(SegView v, int nsys) {
  __shared__ int any[256];
  int open = 0;
  for (int s = threadIdx.x; s < nsys; s += 256) open |= v.done[s] == 0;
  any[threadIdx.x] = open;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (int(threadIdx.x) < off) any[threadIdx.x] |= any[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) v.done[nsys] = any[0] ? 0 : 1;
}

// compact status record per system: (m, reason, eps)
__global__ void lz_status_batched(SegView v, int nsys, LzStatus *__restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys) return;
  out[s].m = v.st[s].m;
  out[s].reason = v.st[s].reason;
  out[s].eps = v.st[s].eps;
}

// y = x / s, or x /= s in place when y == x (square-root preconditioning)
__global__ void divide_by(int64_t m, const double *__restrict__ x, const double *__restrict__ s,
                          double *y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < m) y[i] = x[i] / s[i];
}

__global__ void multiply_by(int64_t m, double *x, const double *__restrict__ s) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < m) x[i] *= s[i];
}

inline unsigned nblk(int64_t m) { return unsigned((m + kThreads - 1) / kThreads); }


int dot(rpb_ctx *ctx, int64_t m, const double *a, const double *b, double *part, double *out,
        int mode, hipStream_t stream) {
  dot_partial<<<kRedBlocks, kThreads, 0, stream>>>(m, a, b, part);
  RPB_LAUNCHED(ctx);
  dot_finish<<<1, kThreads, 0, stream>>>(part, kRedBlocks, out, mode);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

}  // namespace

// One eigensolve of the second stream: wait for iteration k's vector work (event
// lz_vec_ev[slot]), the eigensolve and stop test (lanczos_eig), then the status event of ring
// slot `slot` (lz_ev[slot]).
struct LzJob {
  void *ls;          // LzState
  void *eig;         // LzEig
  void *ring_slot;   // LzRingSlot, device address
  int k;
  double tol;
  int slot;
};

// The second stream's host calls of the small-system solves, issued by a thread of its own:
// a cross-stream wait, a launch and an event record take ~15 us of host time per iteration,
// which the calling thread spends on the next iteration's launches instead (the two threads'
// calls overlap).  Jobs are issued in the order they are queued; `posted` counts those whose
// calls have been issued (their status event then exists).
struct LzHelper {
  std::thread th;
  std::mutex mu;
  std::condition_variable cv_job, cv_done;
  std::deque<LzJob> jobs;
  int64_t pushed = 0, posted = 0;
  bool stop = false;
  hipError_t err = hipSuccess;   // the first failed call, reported to the caller by lz_helper_wait
  const char *what = nullptr;
};

namespace {

void lz_helper_run(rpb_ctx *ctx, LzHelper *h) {
  (void)hipSetDevice(ctx->device);
  for (;;) {
    LzJob j;
    {
      std::unique_lock<std::mutex> lk(h->mu);
      h->cv_job.wait(lk, [&] { return h->stop || !h->jobs.empty(); });
      if (h->jobs.empty()) return;   // stopped with nothing left to issue
      j = h->jobs.front();
      h->jobs.pop_front();
    }
    const char *what = "hipStreamWaitEvent";
    hipError_t e = hipStreamWaitEvent(ctx->lz_stream, ctx->lz_vec_ev[j.slot], 0);
    if (e == hipSuccess) {
      lanczos_eig<<<1, kThreads, 0, ctx->lz_stream>>>(static_cast<LzState *>(j.ls),
                                                      static_cast<LzEig *>(j.eig), j.k, j.tol,
                                                      static_cast<LzRingSlot *>(j.ring_slot));
      e = hipGetLastError();
      what = "lanczos_eig launch";
    }
    if (e == hipSuccess) {
      e = hipEventRecord(ctx->lz_ev[j.slot], ctx->lz_stream);
      what = "hipEventRecord";
    }
    {
      std::lock_guard<std::mutex> lk(h->mu);
      if (e != hipSuccess && h->err == hipSuccess) {
        h->err = e;
        h->what = what;
      }
      ++h->posted;
    }
    h->cv_done.notify_all();
  }
}

// The context's helper, started on first use (with the ring's status events).
int lz_helper_get(rpb_ctx *ctx, LzHelper **out) {
  if (!ctx->lz_helper) {
    for (auto &e : ctx->lz_ev)
      if (!e) RPB_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    LzHelper *h = new (std::nothrow) LzHelper();
    if (!h) return fail(ctx, RPB_ENOMEM, "no memory for the Lanczos helper");
    try {
      h->th = std::thread(lz_helper_run, ctx, h);
    } catch (...) {
      delete h;
      return fail(ctx, RPB_EDEVICE, "could not start the Lanczos helper thread");
    }
    ctx->lz_helper = h;
  }
  *out = ctx->lz_helper;
  return RPB_OK;
}

// Queues a job; returns its sequence number.
int64_t lz_helper_push(LzHelper *h, const LzJob &j) {
  int64_t seq;
  {
    std::lock_guard<std::mutex> lk(h->mu);
    h->jobs.push_back(j);
    seq = ++h->pushed;
  }
  h->cv_job.notify_one();
  return seq;
}

// Blocks until the jobs up to sequence number `seq` are issued; reports a failed call.
int lz_helper_wait(rpb_ctx *ctx, LzHelper *h, int64_t seq) {
  hipError_t e;
  const char *what;
  {
    std::unique_lock<std::mutex> lk(h->mu);
    h->cv_done.wait(lk, [&] { return h->posted >= seq; });
    e = h->err;
    what = h->what;
    h->err = hipSuccess;
  }
  if (e != hipSuccess)
    return fail(ctx, RPB_EDEVICE, "%s failed: %s (Lanczos helper)", what, hipGetErrorString(e));
  return RPB_OK;
}

}  // namespace

void lz_helper_destroy(rpb_ctx *ctx) {
  LzHelper *h = ctx->lz_helper;
  if (!h) return;
  {
    std::lock_guard<std::mutex> lk(h->mu);
    h->stop = true;
  }
  h->cv_job.notify_all();
  if (h->th.joinable()) h->th.join();
  delete h;
  ctx->lz_helper = nullptr;
}

int lanczos_run(rpb_ctx *ctx, const rpb_params *p, const Packed &g, const double *w, double tol,
                int max_iter, bool precond, double *out, int *iters, double *eps_out,
                hipStream_t stream, const double *mw) {
  const int64_t n = g.n;
  const int64_t m3 = 3 * n;
  int st;
  double *L = nullptr, *t = nullptr;
  if (precond) {
    L = static_cast<double *>(workspace(ctx, WS_PRECOND, size_t(2 * m3) * sizeof(double), &st));
    if (!L) return st;
    t = L + m3;
    RPB_TRY(block_diag_scale(ctx, p, g, L, stream));
  }
  double *V = static_cast<double *>(
      workspace(ctx, WS_KRYLOV, size_t(max_iter) * size_t(m3) * sizeof(double), &st));
  if (!V) return st;
  double *u = static_cast<double *>(workspace(ctx, WS_VEC_A, size_t(m3) * sizeof(double), &st));
  if (!u) return st;
  double *part = static_cast<double *>(
      workspace(ctx, WS_REDUCE, size_t(kRedBlocks) * (kMaxKrylov + 1) * sizeof(double), &st));
  if (!part) return st;
  LzState *ls = static_cast<LzState *>(workspace(ctx, WS_SMALL, kSmallBytes, &st));
  if (!ls) return st;
  LzEig *eig = static_cast<LzEig *>(workspace(ctx, WS_LZEIG, sizeof(LzEig), &st));
  if (!eig) return st;
  // The host reads the status of iteration m only after iterations up to m + lag have been
  // enqueued, so the device never idles while the host decides.  Small systems (one workgroup
  // per iteration) run the eigensolve and stop test of iteration k on a second stream beside
  // the product of iteration k + 1 (lag 2); larger ones keep them in line on `stream` (lag 1),
  // where an iteration the stop test has not yet cleared would cost a whole product.  Every
  // kernel of an iteration past the stop leaves the result unchanged: it touches only u, h,
  // V's next column, the packed sources of the next product, entries of alpha and beta past
  // the last iteration and, once the stop is seen, the skip flag of the products (which then
  // return at once); the eigensolve is skipped (y, eps and reason stay).
  RPB_TRY(lz_ring_fence(ctx));
  LzRing *ring = lz_ring(ctx);
  LzRing *ring_dev = lz_ring_dev(ctx);
  const bool fused = m3 <= kFusedSegment;
  // without the preconditioner the kernel that forms v_{k+1} also packs it for the next product
  // (lanczos_vec, or scale_by_inverse_packed for larger systems)
  const bool prepack = !precond;
  void *src = nullptr;
  if (prepack) {
    src = source_buffer(ctx, g, &st);
    if (!src) return st;
  }
  const double *hw = prepack ? packed_weights(g) : nullptr;
  const bool f64 = g.precision == RPB_FP64;
  hipStream_t es = ctx->lz_stream;
  LzHelper *helper = nullptr;   // issues the second stream's calls (small systems)
  if (fused) RPB_TRY(lz_helper_get(ctx, &helper));
  int64_t seq[kLzRing] = {};    // helper job of the iteration in each ring slot
  int64_t last_seq = 0;
  const int lag = fused ? 2 : 1;
  const int *stopped = fused ? &ls->halt : &ls->reason;

  lz_reset<<<1, 64, 0, stream>>>(ls);
  RPB_LAUNCHED(ctx);
  RPB_TRY(dot(ctx, m3, w, w, part, &ls->wnorm, 1, stream));
  scale_by_inverse<<<nblk(m3), kThreads, 0, stream>>>(m3, w, &ls->wnorm, V, nullptr);
  RPB_LAUNCHED(ctx);

  int m = 0;           // iterations whose result counts
  int reason = 0;
  double eps = 0.0;
  size_t mark[kLzRing] = {};   // first timing record of each iteration in flight
  bool stop = false;
  int next_q = 1;      // first iteration whose status the host has not read
  auto iterate = [&]() -> int {
    for (int k = 1; k <= max_iter && !stop; ++k) {
      const int slot = k % kLzRing;
      mark[slot] = ctx->ev_start.size();
      double *vm = V + int64_t(k - 1) * m3;
      const double *vprev = k > 1 ? V + int64_t(k - 2) * m3 : nullptr;
      if (precond) {   // u = L^-1 M L^-1 vm
        divide_by<<<nblk(m3), kThreads, 0, stream>>>(m3, vm, L, t);
        RPB_LAUNCHED(ctx);
        RPB_TRY(matvec_packed(ctx, p, g, t, nullptr, 0, n, u, stream, stopped));
        divide_by<<<nblk(m3), kThreads, 0, stream>>>(m3, u, L, u);
        RPB_LAUNCHED(ctx);
      } else if (k == 1 && mw) {   // M v_1 = (M w) / |w| from the caller's product
        scale_by_inverse<<<nblk(m3), kThreads, 0, stream>>>(m3, mw, &ls->wnorm, u, nullptr);
        RPB_LAUNCHED(ctx);
      } else if (prepack && k > 1) {   // v_k packed by the previous iteration's lanczos_vec
        RPB_TRY(matvec_prepacked(ctx, p, g, src, u, stream, stopped));
      } else {
        RPB_TRY(matvec_packed(ctx, p, g, vm, nullptr, 0, n, u, stream, stopped));
      }
      if (fused) {   // the vector work in one workgroup; the eigensolve on the second stream
        if (f64)
          lanczos_vec<double><<<1, kThreads, 0, stream>>>(
              ls, V, u, m3, k, k < max_iter, hw, static_cast<double *>(src));
        else
          lanczos_vec<float><<<1, kThreads, 0, stream>>>(
              ls, V, u, m3, k, k < max_iter, hw, static_cast<float *>(src));
        RPB_LAUNCHED(ctx);
        RPB_HIP(ctx, hipEventRecord(ctx->lz_vec_ev[slot], stream));
        ctx->lz_live[slot] = true;   // the helper records lz_ev[slot] after its eigensolve
        seq[slot] = last_seq =
            lz_helper_push(helper, LzJob{ls, eig, &ring_dev->slot[slot], k, tol, slot});
      } else {   // six kernels (see dot_partial)
        double *apart = part + int64_t(kRedBlocks) * kMaxKrylov;   // partials of v_k . u
        dot_partial<<<kRedBlocks, kThreads, 0, stream>>>(m3, vm, u, apart);
        RPB_LAUNCHED(ctx);
        const dim3 grid{unsigned(kRedBlocks), unsigned(k), 1u};
        reorth_dots_3t<<<grid, kThreads, 0, stream>>>(m3, V, u, vm, vprev, apart, kRedBlocks,
                                                       &ls->alpha[k - 1],
                                                       k > 1 ? &ls->beta[k - 2] : nullptr, part);
        RPB_LAUNCHED(ctx);
        reorth_finish<<<unsigned(k), kThreads, 0, stream>>>(kRedBlocks, part, ls->h);
        RPB_LAUNCHED(ctx);
        reorth_update_sq<<<kRedBlocks, kThreads, 0, stream>>>(m3, k, V, u, vm, vprev, ls, part);
        RPB_LAUNCHED(ctx);
        beta_eig<<<1, kThreads, 0, stream>>>(kRedBlocks, part, k, tol, ls, eig,
                                             &ring_dev->slot[slot]);
        RPB_LAUNCHED(ctx);
        if (k < max_iter) {
          double *next = V + int64_t(k) * m3;
          if (!prepack)
            scale_by_inverse<<<nblk(m3), kThreads, 0, stream>>>(m3, u, &ls->beta[k - 1], next,
                                                                 ls);
          else if (f64)
            scale_by_inverse_packed<double><<<nblk(m3), kThreads, 0, stream>>>(
                m3, u, &ls->beta[k - 1], next, ls, hw, static_cast<double *>(src));
          else
            scale_by_inverse_packed<float><<<nblk(m3), kThreads, 0, stream>>>(
                m3, u, &ls->beta[k - 1], next, ls, hw, static_cast<float *>(src));
          RPB_LAUNCHED(ctx);
        }
        RPB_TRY(lz_ring_post(ctx, slot, stream));
      }
      // the statuses up to iteration k - lag (all of them after the last iteration)
      const int qmax = k < max_iter ? k - lag : k;
      for (; next_q <= qmax; ++next_q) {
        const int q = next_q;
        if (fused) RPB_TRY(lz_helper_wait(ctx, helper, seq[q % kLzRing]));
        RPB_TRY(lz_ring_wait(ctx, q % kLzRing));
        m = q;
        reason = ring->slot[q % kLzRing].reason;
        eps = ring->slot[q % kLzRing].eps;
        if (reason != 0) {
          // the iterations after q did no work that counts: drop their pair-kernel timing
          // records (some may have run in full before the stop was seen, others not at all)
          if (q < k) timing_discard(ctx, mark[(q + 1) % kLzRing]);
          stop = true;
          break;
        }
      }
    }
    return RPB_OK;
  };
  int status = iterate();
  if (fused) {   // the second stream's work, all of it, before anything later on `stream`
    const int hs = lz_helper_wait(ctx, helper, last_seq);
    if (status == RPB_OK) status = hs;
    RPB_HIP(ctx, hipEventRecord(ctx->lz_join_ev, es));
    RPB_HIP(ctx, hipStreamWaitEvent(stream, ctx->lz_join_ev, 0));
  }
  if (status != RPB_OK) return status;
  basis_combine<<<nblk(m3), kThreads, 0, stream>>>(m3, m, V, ls->y, out);
  RPB_LAUNCHED(ctx);
  if (precond) {
    multiply_by<<<nblk(m3), kThreads, 0, stream>>>(m3, out, L);
    RPB_LAUNCHED(ctx);
  }
  if (iters) *iters = m;
  if (eps_out) *eps_out = eps;
  if (reason == 4) return fail(ctx, RPB_EDEVICE, "tridiagonal eigensolve did not converge");
  if (reason == 3) return fail(ctx, RPB_ENOTSPD, "negative Ritz value at m = %d", m);
  if (reason == 0)
    return fail(ctx, RPB_ENOCONV, "Lanczos: eps = %.3e > tol = %.3e after %d iterations", eps,
                tol, m);
  return RPB_OK;
}


namespace {

// One Krylov process per segment (system) of `b`; product(src, done_dev, done_host, dst) writes
// dst = M src for every segment not yet done (done_host: the flags as of the last host read,
// NULL when unknown).  L (nullable): preconditioner scale, 3 b.n entries, with scratch t.
// mw (nullable, not with L): M w computed by the caller, used for the first iteration.
template <typename Product>
int lanczos_segments(rpb_ctx *ctx, const Batch &b, const double *L, double *t, const double *w,
                     double tol, int max_iter, Product &&product, double *out, bool sync_each,
                     LzStatus *status_host, hipStream_t stream, const double *mw = nullptr) {
  const int64_t m3 = 3 * b.n;
  const int nsys = b.nsys;
  int st;
  double *V = static_cast<double *>(
      workspace(ctx, WS_KRYLOV, size_t(max_iter) * size_t(m3) * sizeof(double), &st));
  if (!V) return st;
  double *u = static_cast<double *>(workspace(ctx, WS_VEC_A, size_t(m3) * sizeof(double), &st));
  if (!u) return st;
  double *part = static_cast<double *>(workspace(
      ctx, WS_REDUCE, size_t(nsys) * kMaxKrylov * kSegBlocks * sizeof(double), &st));
  if (!part) return st;
  const size_t states_bytes = size_t(nsys) * sizeof(LzState);
  const size_t status_off = (states_bytes + size_t(nsys + 1) * sizeof(int) + 255) / 256 * 256;
  char *lz = static_cast<char *>(
      workspace(ctx, WS_LZBATCH, status_off + size_t(nsys) * sizeof(LzStatus), &st));
  if (!lz) return st;
  LzEig *eig = static_cast<LzEig *>(workspace(ctx, WS_LZEIG, size_t(nsys) * sizeof(LzEig), &st));
  if (!eig) return st;
  SegView v{b.offs, b.sys_of, reinterpret_cast<LzState *>(lz),
            reinterpret_cast<int *>(lz + states_bytes), eig};
  LzStatus *status_dev = reinterpret_cast<LzStatus *>(lz + status_off);
  const unsigned ns = unsigned(nsys);
  const int f_alpha = int(offsetof(LzState, alpha) / sizeof(double));
  const int f_beta = int(offsetof(LzState, beta) / sizeof(double));
  const int f_wnorm = int(offsetof(LzState, wnorm) / sizeof(double));
  auto seg_dot = [&](const double *a, const double *c, int field, int mode) -> int {
    seg_dot_partial<<<dim3{unsigned(kSegBlocks), ns, 1u}, kThreads, 0, stream>>>(v, a, c, part);
    RPB_LAUNCHED(ctx);
    seg_dot_finish<<<ns, 64, 0, stream>>>(v, part, field, mode);
    RPB_LAUNCHED(ctx);
    return RPB_OK;
  };

  lz_reset_batched<<<ns, 64, 0, stream>>>(v, nsys);
  RPB_LAUNCHED(ctx);
  RPB_TRY(seg_dot(w, w, f_wnorm, 1));
  seg_scale_by_inverse<<<nblk(m3), kThreads, 0, stream>>>(v, m3, w, f_wnorm, V);
  RPB_LAUNCHED(ctx);
  int *host_done = static_cast<int *>(host_scratch(ctx));
  const int *known = nullptr;   // host copy of the flags, once read
  bool fused = true;            // every system small enough for one workgroup per iteration
  for (int s = 0; s < nsys; ++s)
    fused = fused && 3 * (b.host_offs[s + 1] - b.host_offs[s]) <= kFusedSegment;
  for (int k = 1; k <= max_iter; ++k) {
    double *vk = V + int64_t(k - 1) * m3;
    const double *vprev = k > 1 ? V + int64_t(k - 2) * m3 : nullptr;
    if (L) {   // u = L^-1 M L^-1 vk (rows of finished systems are not used)
      divide_by<<<nblk(m3), kThreads, 0, stream>>>(m3, vk, L, t);
      RPB_LAUNCHED(ctx);
      RPB_TRY(product(t, v.done, known, u));
      divide_by<<<nblk(m3), kThreads, 0, stream>>>(m3, u, L, u);
      RPB_LAUNCHED(ctx);
    } else if (k == 1 && mw) {   // M v_1 = (M w) / |w| per system, from the caller's product
      seg_scale_by_inverse<<<nblk(m3), kThreads, 0, stream>>>(v, m3, mw, f_wnorm, u);
      RPB_LAUNCHED(ctx);
    } else {
      RPB_TRY(product(vk, v.done, known, u));
    }
    if (fused) {   // every system's iteration in one workgroup
      seg_lanczos_step<<<ns, kThreads, 0, stream>>>(v, V, u, m3, k, tol, k < max_iter);
      RPB_LAUNCHED(ctx);
      seg_all_done<<<1, 256, 0, stream>>>(v, nsys);
      RPB_LAUNCHED(ctx);
    } else {
      RPB_TRY(seg_dot(vk, u, f_alpha + k - 1, 0));
      seg_reorth_dots_3t<<<dim3{unsigned(kSegBlocks), unsigned(k), ns}, kThreads, 0, stream>>>(
          v, m3, k, V, u, vk, vprev, part);
      RPB_LAUNCHED(ctx);
      seg_reorth_finish<<<ns, 64, 0, stream>>>(v, k, part);
      RPB_LAUNCHED(ctx);
      seg_reorth_update_sq<<<dim3{unsigned(kSegBlocks), ns, 1u}, kThreads, 0, stream>>>(
          v, m3, k, V, u, vk, vprev, part);
      RPB_LAUNCHED(ctx);
      seg_beta_eig<<<ns, 64, 0, stream>>>(v, k, tol, part);
      RPB_LAUNCHED(ctx);
      seg_all_done<<<1, 256, 0, stream>>>(v, nsys);
      RPB_LAUNCHED(ctx);
      if (k < max_iter) {
        seg_scale_by_inverse<<<nblk(m3), kThreads, 0, stream>>>(v, m3, u, f_beta + k - 1,
                                                                 V + int64_t(k) * m3);
        RPB_LAUNCHED(ctx);
      }
    }
    if (sync_each) {
      RPB_HIP(ctx, hipMemcpyAsync(host_done, v.done, size_t(nsys) * sizeof(int),
                                  hipMemcpyDeviceToHost, stream));
      RPB_HIP(ctx, hipStreamSynchronize(stream));
      bool all = true;
      for (int s = 0; s < nsys && all; ++s) all = host_done[s] != 0;
      if (all) break;
      known = host_done;
    }
  }
  seg_basis_combine<<<nblk(m3), kThreads, 0, stream>>>(v, m3, V, out);
  RPB_LAUNCHED(ctx);
  if (L) {
    multiply_by<<<nblk(m3), kThreads, 0, stream>>>(m3, out, L);
    RPB_LAUNCHED(ctx);
  }
  lz_status_batched<<<(ns + 63) / 64, 64, 0, stream>>>(v, nsys, status_dev);
  RPB_LAUNCHED(ctx);
  if (status_host) {
    RPB_HIP(ctx, hipMemcpyAsync(status_host, status_dev, size_t(nsys) * sizeof(LzStatus),
                                hipMemcpyDeviceToHost, stream));
    RPB_HIP(ctx, hipStreamSynchronize(stream));
  }
  return RPB_OK;
}

}  // namespace

int lanczos_batched_run(rpb_ctx *ctx, const rpb_params *p, const Batch &b, const Packed &g,
                        const double *w, double tol, int max_iter, bool precond, double *out,
                        bool sync_each, LzStatus *status_host, hipStream_t stream,
                        const double *mw) {
  const int64_t m3 = 3 * b.n;
  double *L = nullptr, *t = nullptr;
  if (precond) {
    int st;
    L = static_cast<double *>(workspace(ctx, WS_PRECOND, size_t(2 * m3) * sizeof(double), &st));
    if (!L) return st;
    t = L + m3;
    RPB_TRY(block_diag_scale(ctx, p, g, L, stream));
  }
  auto product = [&](const double *src, const int *done_dev, const int *, double *dst) {
    return matvec_batched(ctx, p, b, g, src, nullptr, done_dev, dst, stream);
  };
  return lanczos_segments(ctx, b, L, t, w, tol, max_iter, product, out, sync_each, status_host,
                          stream, precond ? nullptr : mw);
}

int lanczos_batched_status_copy(rpb_ctx *ctx, int nsys, LzStatus *host, hipStream_t stream) {
  const size_t states_bytes = size_t(nsys) * sizeof(LzState);
  const size_t status_off = (states_bytes + size_t(nsys + 1) * sizeof(int) + 255) / 256 * 256;
  const DevBuf &b = ctx->ws[WS_LZBATCH];
  if (!b.ptr || b.bytes < status_off + size_t(nsys) * sizeof(LzStatus))
    return fail(ctx, RPB_EINVAL, "no batched Lanczos state");
  RPB_HIP(ctx, hipMemcpyAsync(host, static_cast<char *>(b.ptr) + status_off,
                              size_t(nsys) * sizeof(LzStatus), hipMemcpyDeviceToHost, stream));
  RPB_HIP(ctx, hipStreamSynchronize(stream));
  return RPB_OK;
}

int lanczos_status_code(rpb_ctx *ctx, const LzStatus *s, int nsys) {
  int worst = RPB_OK;
  for (int q = 0; q < nsys; ++q) {
    if (s[q].reason == 4)
      return fail(ctx, RPB_EDEVICE, "tridiagonal eigensolve failed (system %d)", q);
    if (s[q].reason == 3) worst = fail(ctx, RPB_ENOTSPD, "negative Ritz value (system %d)", q);
    if (s[q].reason == 0 && worst == RPB_OK)
      worst = fail(ctx, RPB_ENOCONV, "Lanczos tolerance not met (system %d, eps %.3e)", q,
                   s[q].eps);
  }
  return worst;
}

}  // namespace rpb

using namespace rpb;

namespace {

int lanczos_entry(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                  const double *w, double tol, int max_iter, bool precond, double *out,
                  int *iters_out, double *eps_out, rpb_stream_t stream_) {
  RPB_TRY(check_params(ctx, p));
  if (n < 0) return fail(ctx, RPB_EINVAL, "n must be >= 0");
  if (!(tol > 0.0)) return fail(ctx, RPB_EINVAL, "tol must be > 0");
  if (max_iter < 1 || max_iter > kMaxKrylov)
    return fail(ctx, RPB_EINVAL, "max_iter must be in [1, %d]", kMaxKrylov);
  if (iters_out) *iters_out = 0;
  if (eps_out) *eps_out = 0.0;
  if (n == 0) return RPB_OK;
  if (!pos || !w || !out) return fail(ctx, RPB_EINVAL, "pos, w and out must not be NULL");
  const size_t nb = size_t(n) * 3 * sizeof(double);
  if (overlaps(out, nb, pos, nb) || overlaps(out, nb, w, nb))
    return fail(ctx, RPB_EINVAL, "out overlaps an input");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  RPB_HIP(ctx, hipSetDevice(ctx->device));
  RPB_TRY(check_finite(ctx, pos, n, stream));
  Packed g;
  RPB_TRY(pack_geometry(ctx, p, n, pos, WS_GEOM, &g, stream));
  const int lz =
      lanczos_run(ctx, p, g, w, tol, max_iter, precond, out, iters_out, eps_out, stream);
  if (lz != RPB_OK && lz != RPB_ENOCONV) return lz;
  RPB_TRY(check_output(ctx, out, 3 * n, stream, "the Brownian increment"));
  return lz;
}

}  // namespace

extern "C" int lanczos_sqrt_apply(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                                  const double *w, double tol, int max_iter, double *out,
                                  int *iters_out, double *eps_out, rpb_stream_t stream) {
  return lanczos_entry(ctx, p, n, pos, w, tol, max_iter, false, out, iters_out, eps_out, stream);
}

extern "C" int lanczos_sqrt_apply_precond(rpb_ctx *ctx, const rpb_params *p, int64_t n,
                                          const double *pos, const double *w, double tol,
                                          int max_iter, double *out, int *iters_out,
                                          double *eps_out, rpb_stream_t stream) {
  return lanczos_entry(ctx, p, n, pos, w, tol, max_iter, true, out, iters_out, eps_out, stream);
}

extern "C" int lanczos_sqrt_apply_batched(rpb_ctx *ctx, const rpb_params *p, int32_t nsys,
                                          const int64_t *offs, const double *pos,
                                          const double *w, double tol, int max_iter, double *out,
                                          int *iters_out, double *eps_out, rpb_stream_t stream_) {
  RPB_TRY(check_params(ctx, p));
  RPB_TRY(check_offsets(ctx, nsys, offs));
  if (p->lx > 0.0)
    return fail(ctx, RPB_EINVAL, "pseudo-periodic boundaries are supported for single systems");
  if (nsys > kMaxBatchSystems)
    return fail(ctx, RPB_EINVAL, "at most %d systems per batch", kMaxBatchSystems);
  if (!(tol > 0.0)) return fail(ctx, RPB_EINVAL, "tol must be > 0");
  if (max_iter < 1 || max_iter > kMaxKrylov)
    return fail(ctx, RPB_EINVAL, "max_iter must be in [1, %d]", kMaxKrylov);
  const int64_t n = offs[nsys];
  for (int s = 0; s < nsys; ++s) {
    if (iters_out) iters_out[s] = 0;
    if (eps_out) eps_out[s] = 0.0;
  }
  if (n == 0) return RPB_OK;
  if (!pos || !w || !out) return fail(ctx, RPB_EINVAL, "pos, w and out must not be NULL");
  const size_t nb = size_t(n) * 3 * sizeof(double);
  if (overlaps(out, nb, pos, nb) || overlaps(out, nb, w, nb))
    return fail(ctx, RPB_EINVAL, "out overlaps an input");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  RPB_HIP(ctx, hipSetDevice(ctx->device));
  RPB_TRY(check_finite(ctx, pos, n, stream));
  Batch b;
  RPB_TRY(prepare_batch(ctx, nsys, offs, p->precision, &b, stream));
  Packed g;
  RPB_TRY(pack_geometry(ctx, p, n, pos, WS_GEOM, &g, stream));
  LzStatus *stat = static_cast<LzStatus *>(host_scratch(ctx));
  RPB_TRY(lanczos_batched_run(ctx, p, b, g, w, tol, max_iter, false, out, true, stat, stream));
  for (int s = 0; s < nsys; ++s) {
    if (iters_out) iters_out[s] = stat[s].m;
    if (eps_out) eps_out[s] = stat[s].eps;
  }
  return lanczos_status_code(ctx, stat, nsys);
}

extern "C" int lanczos_sqrt_apply_multi(rpb_ctx *ctx, const rpb_params *p, int64_t n,
                                        const double *pos, int32_t nvec, const double *w,
                                        double tol, int max_iter, double *out, int *iters_out,
                                        double *eps_out, rpb_stream_t stream_) {
  RPB_TRY(check_params(ctx, p));
  if (n < 0) return fail(ctx, RPB_EINVAL, "n must be >= 0");
  if (nvec < 0 || nvec > kMaxBatchSystems)
    return fail(ctx, RPB_EINVAL, "nvec must be in [0, %d]", kMaxBatchSystems);
  if (p->lx > 0.0)
    return fail(ctx, RPB_EINVAL, "pseudo-periodic boundaries are not supported for "
                                 "multi-vector products");
  if (!(tol > 0.0)) return fail(ctx, RPB_EINVAL, "tol must be > 0");
  if (max_iter < 1 || max_iter > kMaxKrylov)
    return fail(ctx, RPB_EINVAL, "max_iter must be in [1, %d]", kMaxKrylov);
  for (int s = 0; s < nvec; ++s) {
    if (iters_out) iters_out[s] = 0;
    if (eps_out) eps_out[s] = 0.0;
  }
  if (n == 0 || nvec == 0) return RPB_OK;
  if (!pos || !w || !out) return fail(ctx, RPB_EINVAL, "pos, w and out must not be NULL");
  const size_t pb = size_t(n) * 3 * sizeof(double), vb = pb * size_t(nvec);
  if (overlaps(out, vb, pos, pb) || overlaps(out, vb, w, vb))
    return fail(ctx, RPB_EINVAL, "out overlaps an input");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  RPB_HIP(ctx, hipSetDevice(ctx->device));
  RPB_TRY(check_finite(ctx, pos, n, stream));
  // vector v is segment v of a batch of nvec segments of n spheres each
  std::vector<int64_t> offs(size_t(nvec) + 1);
  for (int s = 0; s <= nvec; ++s) offs[size_t(s)] = int64_t(s) * n;
  Batch b;
  RPB_TRY(prepare_batch(ctx, nvec, offs.data(), p->precision, &b, stream, false));
  Packed g;
  RPB_TRY(pack_geometry(ctx, p, n, pos, WS_GEOM, &g, stream));
  auto product = [&](const double *src, const int *, const int *done_host, double *dst) {
    return matvec_multi(ctx, p, g, nvec, done_host, src, dst, stream);
  };
  LzStatus *stat = static_cast<LzStatus *>(host_scratch(ctx));
  RPB_TRY(lanczos_segments(ctx, b, nullptr, nullptr, w, tol, max_iter, product, out, true, stat,
                           stream));
  for (int s = 0; s < nvec; ++s) {
    if (iters_out) iters_out[s] = stat[s].m;
    if (eps_out) eps_out[s] = stat[s].eps;
  }
  return lanczos_status_code(ctx, stat, nvec);
}

extern "C" int lanczos_tridiag_sqrt(rpb_ctx *ctx, int32_t m, const double *alpha,
                                    const double *beta, double wnorm, double *y_out,
                                    rpb_stream_t stream_) {
  if (!ctx) return RPB_EINVAL;
  if (m < 1 || m > kMaxKrylov) return fail(ctx, RPB_EINVAL, "m must be in [1, %d]", kMaxKrylov);
  if (!alpha || (m > 1 && !beta) || !y_out)
    return fail(ctx, RPB_EINVAL, "alpha, beta and y_out must not be NULL");
  if (!std::isfinite(wnorm) || wnorm < 0.0)
    return fail(ctx, RPB_EINVAL, "wnorm must be finite and >= 0");
  LzState h{};
  for (int i = 0; i < m; ++i) {
    if (!std::isfinite(alpha[i]) || (i < m - 1 && !std::isfinite(beta[i])))
      return fail(ctx, RPB_EINVAL, "alpha and beta must be finite");
    h.alpha[i] = alpha[i];
    if (i < m - 1) h.beta[i] = beta[i];
  }
  h.wnorm = wnorm;
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  RPB_HIP(ctx, hipSetDevice(ctx->device));
  int st;
  LzState *ls = static_cast<LzState *>(workspace(ctx, WS_SMALL, kSmallBytes, &st));
  if (!ls) return st;
  LzEig *eig = static_cast<LzEig *>(workspace(ctx, WS_LZEIG, sizeof(LzEig), &st));
  if (!eig) return st;
  const size_t ybytes = size_t(m) * size_t(m) * sizeof(double);
  char *buf = static_cast<char *>(workspace(ctx, WS_VEC_A, ybytes + sizeof(int), &st));
  if (!buf) return st;
  int *flag = reinterpret_cast<int *>(buf + ybytes);
  RPB_HIP(ctx, hipMemcpyAsync(ls, &h, sizeof(LzState), hipMemcpyHostToDevice, stream));
  tridiag_sequence<<<1, 64, 0, stream>>>(m, ls, eig, reinterpret_cast<double *>(buf), flag);
  RPB_LAUNCHED(ctx);
  int failed = 0;
  RPB_HIP(ctx, hipMemcpyAsync(y_out, buf, ybytes, hipMemcpyDeviceToHost, stream));
  RPB_HIP(ctx, hipMemcpyAsync(&failed, flag, sizeof(int), hipMemcpyDeviceToHost, stream));
  RPB_HIP(ctx, hipStreamSynchronize(stream));
  if (failed) return fail(ctx, RPB_EDEVICE, "tridiagonal eigensolve did not converge");
  return RPB_OK;
}
