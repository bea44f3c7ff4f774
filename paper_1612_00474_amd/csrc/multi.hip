// Products of one configuration's mobility with several source vectors, U_k = M F_k.
//
// The Lanczos method (Sec. IV) needs only products with M, and several independent Krylov
// processes on the same configuration (several noise vectors) need products with the same
// matrix.  The pair coefficients of the regularised Rotne-Prager-Blake tensor (App. A) depend
// on the geometry alone, so one evaluation serves every vector: about half the work of a
// symmetric pair update is the coefficients, the rest is applying them to a vector.
//
// Layout: the symmetric tile-pair scheme of the single-vector product, one target per lane
// (tile = kBlock spheres), kMulti vectors per launch:
//   pack_multi    O(N K)    AoS float64 vectors -> SoA H-weighted sources src[(k 3 + c) n + i]
//   pair kernel   O(N^2)    tile pair (I, J), I <= J, per workgroup: M_IJ F_J into the rows of
//                           I (lane sums), M_JI F_I into the rows of J (rotating per-source sums
//                           added across the workgroup's wavefronts in LDS); diagonal tiles as
//                           ordered pairs.  Each pair's coefficients are computed once.
//   reduce_multi  O(N^2/256) fixed-order sum of the tile partials, times H_i / (8 pi eta).
#include <algorithm>
#include <cmath>
#include <vector>

#include "pair_common.h"

namespace rpb {

namespace {

constexpr int kMulti = 4;            // source vectors per launch (fewer: zero vectors pad)
constexpr int kMultiC = 3 * kMulti;  // source components per sphere
// Largest partial buffer of one launch; larger systems use the single-vector product per vector.
constexpr size_t kMaxMultiPartialBytes = size_t(32) << 30;

struct VecIds {
  int v[kMulti];   // vector of each launch slot, -1 for a zero vector
};

template <typename Real>
__global__ void pack_multi(int64_t n, VecIds ids, const double *__restrict__ h,
                           const double *__restrict__ f, Real *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double w = h[i];
#pragma unroll
  for (int k = 0; k < kMulti; ++k) {
    const int v = ids.v[k];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      out[(k * 3 + c) * n + i] = v >= 0 ? Real(w * f[(int64_t(v) * n + i) * 3 + c]) : Real(0);
  }
}

struct MultiLdsF {
  float xh[kBlock], xl[kBlock], yh[kBlock], yl[kBlock], z[kBlock];
  float f[kMultiC][kBlock];
  float col[kWaves][kMultiC][64];   // per-wavefront sums for one 64-source block
};
struct MultiLdsD {
  double x[kBlock], y[kBlock], z[kBlock];
  double f[kMultiC][kBlock];
  double col[kWaves][kMultiC][64];
};

struct TgtF {
  float xh, xl, yh, yl, z;
};
struct TgtD {
  double x, y, z;
};

__device__ __forceinline__ TgtF target_of(const GeomF &g, int64_t i) {
  return {g.xh[i], g.xl[i], g.yh[i], g.yl[i], g.z[i]};
}
__device__ __forceinline__ TgtD target_of(const GeomD &g, int64_t i) {
  return {g.x[i], g.y[i], g.z[i]};
}
__device__ __forceinline__ void stage(MultiLdsF &L, const GeomF &g, int64_t j, int s) {
  L.xh[s] = g.xh[j];
  L.xl[s] = g.xl[j];
  L.yh[s] = g.yh[j];
  L.yl[s] = g.yl[j];
  L.z[s] = g.z[j];
}
__device__ __forceinline__ void stage(MultiLdsD &L, const GeomD &g, int64_t j, int s) {
  L.x[s] = g.x[j];
  L.y[s] = g.y[j];
  L.z[s] = g.z[j];
}
// In-plane separation r_i - r_j (mixed: hi and lo parts subtracted separately).
__device__ __forceinline__ void separation(const TgtF &t, const MultiLdsF &L, int j, float &dx,
                                           float &dy) {
  dx = (t.xh - L.xh[j]) + (t.xl - L.xl[j]);
  dy = (t.yh - L.yh[j]) + (t.yl - L.yl[j]);
}
__device__ __forceinline__ void separation(const TgtD &t, const MultiLdsD &L, int j, double &dx,
                                           double &dy) {
  dx = t.x - L.x[j];
  dy = t.y - L.y[j];
}

// Coefficients of pair (i, j): the far-field form alone for pairs at least 2a apart, the
// complete form for closer ones (including the self pair, r = 0).
template <bool WALL, typename Real>
__device__ __forceinline__ void multi_coefficients(Real dx, Real dy, Real zi, Real zj,
                                                   const PairConsts<Real> &k, SymCoef<Real> &c) {
  const Real dz = zi - zj;
  if (dx * dx + dy * dy + dz * dz < k.four_a2)
    sym_coefficients<Real, false, false, WALL>(dx, dy, zi, zj, k, c);
  else
    sym_coefficients<Real, true, false, WALL>(dx, dy, zi, zj, k, c);
}

// One rotation step of an off-diagonal tile pair: the lane's target i against source j for
// every vector, M_ij F_j into acc and M_ji F_i into the rotating sums cs (weighted forces zero
// when !valid).
template <bool WALL, typename Real, typename Tgt, typename Lds>
__device__ __forceinline__ void multi_step(const Lds &L, int j, bool valid, const Tgt &t,
                                           const Real (&own)[kMultiC], const PairConsts<Real> &k,
                                           Real (&acc)[kMultiC], Real (&cs)[kMultiC]) {
  Real dx, dy;
  separation(t, L, j, dx, dy);
  const Real zj = L.z[j];
  Real f[kMultiC];
#pragma unroll
  for (int e = 0; e < kMultiC; ++e) f[e] = valid ? L.f[e][j] : Real(0);
#pragma unroll
  for (int e = 0; e < kMultiC; ++e) cs[e] = wave_rol1(cs[e]);
  SymCoef<Real> c;
  multi_coefficients<WALL>(dx, dy, t.z, zj, k, c);
#pragma unroll
  for (int v = 0; v < kMulti; ++v)
    sym_apply<Real, WALL>(c, f[3 * v], f[3 * v + 1], f[3 * v + 2], own[3 * v], own[3 * v + 1],
                          own[3 * v + 2], acc[3 * v], acc[3 * v + 1], acc[3 * v + 2], cs[3 * v],
                          cs[3 * v + 1], cs[3 * v + 2]);
}

// partial[(((v nt + T) nt + P) 3 + comp) kBlock + local]: tile pair (T, P)'s sums for the rows
// of tile T, vector slot v.
__device__ __forceinline__ int64_t multi_slot(const SymArgs &a, int v, int64_t T, int64_t P,
                                              int comp, int64_t local) {
  return (((int64_t(v) * a.nt + T) * a.nt + P) * 3 + comp) * kBlock + local;
}

// Tile pair (I, J), I <= J.  Every lane of the workgroup must call this (it synchronises).
template <bool WALL, typename Real, typename Geom, typename Lds>
__device__ __forceinline__ void multi_tile_pair(const SymArgs &a, const Geom &g,
                                                const Real *__restrict__ src,
                                                const PairConsts<Real> &k,
                                                double *__restrict__ partial, int64_t I,
                                                int64_t J, Lds &L) {
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int64_t n = a.n;
  const int64_t i = I * kBlock + tid;
  const bool on = i < n;
  const auto t = target_of(g, on ? i : I * kBlock);
  const int64_t jb = J * kBlock;
  const int cnt = int(min<int64_t>(kBlock, n - jb));
  if (tid < cnt) {
    stage(L, g, jb + tid, tid);
#pragma unroll
    for (int e = 0; e < kMultiC; ++e) L.f[e][tid] = src[e * a.stride + jb + tid];
  }
  __syncthreads();
  Real acc[kMultiC];
#pragma unroll
  for (int e = 0; e < kMultiC; ++e) acc[e] = Real(0);
  if (I == J) {   // ordered pairs of the diagonal tile, self pair included
    for (int j = 0; j < cnt; ++j) {
      Real dx, dy;
      separation(t, L, j, dx, dy);
      SymCoef<Real> c;
      multi_coefficients<WALL>(dx, dy, t.z, L.z[j], k, c);
#pragma unroll
      for (int v = 0; v < kMulti; ++v)
        sym_apply_one<Real, WALL>(c, L.f[3 * v][j], L.f[3 * v + 1][j], L.f[3 * v + 2][j],
                                  acc[3 * v], acc[3 * v + 1], acc[3 * v + 2]);
    }
  } else {
    Real own[kMultiC];
#pragma unroll
    for (int e = 0; e < kMultiC; ++e) own[e] = on ? src[e * a.stride + i] : Real(0);
    for (int blk = 0; blk < cnt; blk += 64) {
      const int nb = min(64, cnt - blk);
      Real cs[kMultiC];
#pragma unroll
      for (int e = 0; e < kMultiC; ++e) cs[e] = Real(0);
      if (nb == 64) {
        for (int step = 0; step < 64; ++step)
          multi_step<WALL>(L, blk + ((lane + step) & 63), true, t, own, k, acc, cs);
      } else {
        for (int step = 0; step < 64; ++step) {
          const int sl = (lane + step) & 63;
          multi_step<WALL>(L, blk + (sl < nb ? sl : 0), sl < nb, t, own, k, acc, cs);
        }
      }
      // after 64 rotations lane l holds the sums of source (l + 63) mod 64
      const int sl = (lane + 63) & 63;
#pragma unroll
      for (int e = 0; e < kMultiC; ++e) L.col[wave][e][sl] = cs[e];
      __syncthreads();
      for (int e0 = tid; e0 < kMultiC * 64; e0 += kBlock) {
        const int e = e0 / 64, s = e0 % 64;
        if (s < nb) {
          double sum = 0.0;
#pragma unroll
          for (int w = 0; w < kWaves; ++w) sum += double(L.col[w][e][s]);
          partial[multi_slot(a, e / 3, J, I, e % 3, blk + s)] = sum;
        }
      }
      __syncthreads();
    }
  }
  if (on)
#pragma unroll
    for (int e = 0; e < kMultiC; ++e)
      partial[multi_slot(a, e / 3, I, J, e % 3, tid)] = double(acc[e]);
}

template <bool WALL>
__global__ __launch_bounds__(kBlock) void pair_kernel_mixed_multi(SymArgs a, GeomF g,
                                                                  const float *__restrict__ src,
                                                                  PairConsts<float> k,
                                                                  double *__restrict__ partial) {
  __shared__ MultiLdsF L;
  int64_t I, J;
  tri_decode(blockIdx.x, a.nt, I, J);
  multi_tile_pair<WALL>(a, g, src, k, partial, I, J, L);
}

template <bool WALL>
__global__ __launch_bounds__(kBlock) void pair_kernel_f64_multi(SymArgs a, GeomD g,
                                                                const double *__restrict__ src,
                                                                PairConsts<double> k,
                                                                double *__restrict__ partial) {
  __shared__ MultiLdsD L;
  int64_t I, J;
  tri_decode(blockIdx.x, a.nt, I, J);
  multi_tile_pair<WALL>(a, g, src, k, partial, I, J, L);
}

// One thread per (vector slot, component, row); four independent partial sums over the
// slots (P mod 4), combined in a fixed order.
__global__ void reduce_multi(SymArgs a, VecIds ids, const double *__restrict__ partial,
                             const double *__restrict__ h, double scale,
                             double *__restrict__ vel) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = 3 * a.n;
  if (e >= kMulti * per) return;
  const int v = int(e / per);
  const int64_t rem = e - int64_t(v) * per;
  const int d = int(rem / a.n);
  const int64_t r = rem - int64_t(d) * a.n;
  const int id = ids.v[v];
  if (id < 0) return;
  const int64_t T = r / kBlock, local = r % kBlock;
  const double *base = partial + multi_slot(a, v, T, 0, d, local);
  const int64_t stride = 3 * kBlock;   // slot (T, P) to (T, P + 1)
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t P = 0;
  for (; P + 4 <= a.nt; P += 4) {
    s0 += base[P * stride];
    s1 += base[(P + 1) * stride];
    s2 += base[(P + 2) * stride];
    s3 += base[(P + 3) * stride];
  }
  for (; P < a.nt; ++P) s0 += base[P * stride];
  vel[(int64_t(id) * a.n + r) * 3 + d] = scale * h[r] * ((s0 + s1) + (s2 + s3));
}

}  // namespace

int matvec_multi(rpb_ctx *ctx, const rpb_params *p, const Packed &g, int nvec, const int *done,
                 const double *force, double *vel, hipStream_t stream) {
  const int64_t n = g.n;
  if (n == 0 || nvec <= 0) return RPB_OK;
  if (p->lx > 0.0)
    return fail(ctx, RPB_EINVAL, "pseudo-periodic boundaries are not supported for "
                                 "multi-vector products");
  std::vector<int> ids;
  for (int v = 0; v < nvec; ++v)
    if (!done || !done[v]) ids.push_back(v);
  const bool f64 = g.precision == RPB_FP64;
  SymArgs a{n, kBlock, (n + kBlock - 1) / kBlock, n};
  const size_t part_bytes =
      size_t(kMulti) * size_t(a.nt) * size_t(a.nt) * 3 * size_t(kBlock) * sizeof(double);
  if (a.nt * (a.nt + 1) / 2 > 0x7fffffffll || part_bytes > kMaxMultiPartialBytes) {
    // too large for one launch: one single-vector product per vector
    for (int v : ids)
      RPB_TRY(matvec_packed(ctx, p, g, force + size_t(v) * 3 * n, nullptr, 0, n,
                            vel + size_t(v) * 3 * n, stream));
    return RPB_OK;
  }
  int st;
  double *part = static_cast<double *>(workspace(ctx, WS_PART, part_bytes, &st));
  if (!part) return st;
  const size_t esz = f64 ? sizeof(double) : sizeof(float);
  void *src = workspace(ctx, WS_SRC, size_t(kMultiC) * size_t(n) * esz, &st);
  if (!src) return st;
  const double *h = f64 ? geom_d(g).h : geom_f(g).h;
  const unsigned grid = unsigned(a.nt * (a.nt + 1) / 2);
  const double scale = 1.0 / (8.0 * M_PI * p->eta);
  const bool wall = p->wall != 0;
  for (size_t g0 = 0; g0 < ids.size(); g0 += kMulti) {
    VecIds vi;
    int used = 0;
    for (int s = 0; s < kMulti; ++s) {
      vi.v[s] = g0 + s < ids.size() ? ids[g0 + s] : -1;
      used += vi.v[s] >= 0;
    }
    if (f64)
      pack_multi<double><<<blocks_for(n, 256), 256, 0, stream>>>(n, vi, h, force,
                                                                static_cast<double *>(src));
    else
      pack_multi<float><<<blocks_for(n, 256), 256, 0, stream>>>(n, vi, h, force,
                                                               static_cast<float *>(src));
    RPB_LAUNCHED(ctx);
    hipEvent_t t0;
    RPB_TRY(timing_begin(ctx, stream, &t0));
    if (f64) {
      const auto k = make_pair_consts<double>(p->a);
      const auto *s = static_cast<const double *>(src);
      if (wall)
        pair_kernel_f64_multi<true><<<grid, kBlock, 0, stream>>>(a, geom_d(g), s, k, part);
      else
        pair_kernel_f64_multi<false><<<grid, kBlock, 0, stream>>>(a, geom_d(g), s, k, part);
    } else {
      const auto k = make_pair_consts<float>(p->a);
      const auto *s = static_cast<const float *>(src);
      if (wall)
        pair_kernel_mixed_multi<true><<<grid, kBlock, 0, stream>>>(a, geom_f(g), s, k, part);
      else
        pair_kernel_mixed_multi<false><<<grid, kBlock, 0, stream>>>(a, geom_f(g), s, k, part);
    }
    RPB_LAUNCHED(ctx);
    RPB_TRY(timing_end(ctx, stream, t0, double(n) * double(n) * used, 8 + (f64 ? 0 : 2)));
    reduce_multi<<<blocks_for(int64_t(kMulti) * 3 * n, 256), 256, 0, stream>>>(a, vi, part, h,
                                                                               scale, vel);
    RPB_LAUNCHED(ctx);
  }
  return RPB_OK;
}

}  // namespace rpb

using namespace rpb;

extern "C" int rpb_mobility_matvec_multi(rpb_ctx *ctx, const rpb_params *p, int64_t n,
                                         const double *pos, int32_t nvec, const double *force,
                                         double *vel, rpb_stream_t stream_) {
  RPB_TRY(check_params(ctx, p));
  if (n < 0) return fail(ctx, RPB_EINVAL, "n must be >= 0");
  if (nvec < 0) return fail(ctx, RPB_EINVAL, "nvec must be >= 0");
  if (p->lx > 0.0)
    return fail(ctx, RPB_EINVAL, "pseudo-periodic boundaries are not supported for "
                                 "multi-vector products");
  if (n == 0 || nvec == 0) return RPB_OK;
  if (!pos || !force || !vel) return fail(ctx, RPB_EINVAL, "pos, force and vel must not be NULL");
  const size_t pb = size_t(n) * 3 * sizeof(double), vb = pb * size_t(nvec);
  if (overlaps(vel, vb, pos, pb) || overlaps(vel, vb, force, vb))
    return fail(ctx, RPB_EINVAL, "vel overlaps an input");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  RPB_HIP(ctx, hipSetDevice(ctx->device));
  RPB_TRY(check_finite(ctx, pos, n, stream));
  Packed g;
  RPB_TRY(pack_geometry(ctx, p, n, pos, WS_GEOM, &g, stream));
  return matvec_multi(ctx, p, g, nvec, nullptr, force, vel, stream);
}
