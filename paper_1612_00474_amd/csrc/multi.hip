// Products of one configuration's mobility with several source vectors, U_k = M F_k.
//
// The Lanczos method (Sec. II.C) needs only products with M, and several independent Krylov
// processes on the same configuration (several noise vectors) need products with the same
// matrix; so do the products a time step takes at its own configuration (M F + M_C T, the
// first Lanczos product M W and, for a one-sided RFD, M W~).  The pair coefficients of the
// regularised Rotne-Prager-Blake tensor (App. A) depend on the geometry alone, so one
// evaluation serves every vector: about half the work of a symmetric pair update is the
// coefficients, the rest is applying them to a vector.
//
// Layout: the symmetric tile-pair scheme of the single-vector product, one target per lane
// (tile = kBlock spheres), K = 2, 3 or 4 vectors per launch, the first optionally with a torque:
//   pack_multi    O(N K)    AoS float64 vectors -> SoA H-weighted sources src[(k 3 + c) n + i]
//   pair kernel   O(N^2)    tile pair (I, J), I <= J, per workgroup: M_IJ F_J into the rows of
//                           I (lane sums), M_JI F_I into the rows of J (rotating per-source sums
//                           added across the workgroup's wavefronts in LDS); diagonal tiles as
//                           ordered pairs.  Each pair's coefficients are computed once.  Batches
//                           of systems: persistent workgroups map a work-item number to
//                           (system, I, J).
//   reduce_multi  O(N^2/256) fixed-order sum of the tile partials, times H_i / (8 pi eta a).
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "pair_common.h"

namespace rpb {

namespace {

constexpr int kMulti = 4;   // source vectors per launch of the plain multi-vector product
// Partials of one persistent batched launch (every system's triangle at once); larger batches
// take the single-vector batched products.
constexpr size_t kMaxMultiBatchBytes = size_t(4) << 30;

// Source rows of a launch of K vectors: forces of slots 0..K-1 (3 each), then, with TQ, the
// torque of slot 0.
template <int K, bool TQ>
constexpr int src_rows() { return 3 * K + (TQ ? 3 : 0); }

__global__ void zero_counter(int *c) { c[0] = 0; }

template <int K>
struct SrcPtrs {
  const double *p[K];   // [n][3] source vector of each launch slot, NULL for a zero vector
};
template <int K>
struct OutPtrs {
  double *p[K];         // [n][3] result of each slot, NULL: not stored
};

// src[e n + i]: e = 3 k + c holds H_i F_k(i, c); with a torque, e = 3 K + c holds H_i T(i, c)/a
// for slot 0.
template <int K, typename Real>
__global__ void pack_multi(int64_t n, SrcPtrs<K> in, const double *__restrict__ h,
                           const double *__restrict__ torque, double inv_a,
                           Real *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double w = h[i];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double *f = in.p[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) out[(k * 3 + c) * n + i] = f ? Real(w * f[3 * i + c]) : Real(0);
  }
  if (torque)
#pragma unroll
    for (int c = 0; c < 3; ++c) out[(3 * K + c) * n + i] = Real(w * inv_a * torque[3 * i + c]);
}

template <int K, bool TQ>
struct MultiLdsF {
  float xh[kBlock], xl[kBlock], yh[kBlock], yl[kBlock], z[kBlock];
  float f[src_rows<K, TQ>()][kBlock];
  float col[kWaves][3 * K][64];   // per-wavefront sums for one 64-source block
};
template <int K, bool TQ>
struct MultiLdsD {
  double x[kBlock], y[kBlock], z[kBlock];
  double f[src_rows<K, TQ>()][kBlock];
  double col[kWaves][3 * K][64];
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
template <typename Lds>
__device__ __forceinline__ void stage(Lds &L, const GeomF &g, int64_t j, int s) {
  L.xh[s] = g.xh[j];
  L.xl[s] = g.xl[j];
  L.yh[s] = g.yh[j];
  L.yl[s] = g.yl[j];
  L.z[s] = g.z[j];
}
template <typename Lds>
__device__ __forceinline__ void stage(Lds &L, const GeomD &g, int64_t j, int s) {
  L.x[s] = g.x[j];
  L.y[s] = g.y[j];
  L.z[s] = g.z[j];
}
// In-plane separation r_i - r_j (mixed: hi and lo parts subtracted separately).
template <typename Lds>
__device__ __forceinline__ void separation(const TgtF &t, const Lds &L, int j, float &dx,
                                           float &dy) {
  dx = (t.xh - L.xh[j]) + (t.xl - L.xl[j]);
  dy = (t.yh - L.yh[j]) + (t.yl - L.yl[j]);
}
template <typename Lds>
__device__ __forceinline__ void separation(const TgtD &t, const Lds &L, int j, double &dx,
                                           double &dy) {
  dx = t.x - L.x[j];
  dy = t.y - L.y[j];
}

// Coefficients of pair (i, j): the far-field form alone for pairs at least 2a apart, the
// complete form for closer ones (including the self pair, r = 0).
template <bool TQ, bool WALL, typename Real>
__device__ __forceinline__ void multi_coefficients(Real dx, Real dy, Real zi, Real zj,
                                                   const PairConsts<Real> &k, SymCoef<Real> &c) {
  const Real dz = zi - zj;
  if (dx * dx + dy * dy + dz * dz < Real(kFourA2))
    sym_coefficients<Real, false, TQ, WALL>(dx, dy, zi, zj, k, c);
  else
    sym_coefficients<Real, true, TQ, WALL>(dx, dy, zi, zj, k, c);
}

// One rotation step of an off-diagonal tile pair: the lane's target i against source j for
// every vector, M_ij F_j into acc and M_ji F_i into the rotating sums cs (weighted sources
// zero when !valid); with TQ, slot 0 adds the coupling M^C_ij T_j and M^C_ji T_i.
template <int K, bool TQ, bool WALL, typename Real, typename Tgt, typename Lds>
__device__ __forceinline__ void multi_step(const Lds &L, int j, bool valid, const Tgt &t,
                                           const Real (&own)[src_rows<K, TQ>()],
                                           const PairConsts<Real> &k, Real (&acc)[3 * K],
                                           Real (&cs)[3 * K]) {
  constexpr int R = src_rows<K, TQ>();
  Real dx, dy;
  separation(t, L, j, dx, dy);
  const Real zj = L.z[j];
  Real f[R];
#pragma unroll
  for (int e = 0; e < R; ++e) f[e] = valid ? L.f[e][j] : Real(0);
#pragma unroll
  for (int e = 0; e < 3 * K; ++e) cs[e] = wave_rol1(cs[e]);
  SymCoef<Real> c;
  multi_coefficients<TQ, WALL>(dx, dy, t.z, zj, k, c);
#pragma unroll
  for (int v = 0; v < K; ++v)
    sym_apply<Real, WALL>(c, f[3 * v], f[3 * v + 1], f[3 * v + 2], own[3 * v], own[3 * v + 1],
                          own[3 * v + 2], acc[3 * v], acc[3 * v + 1], acc[3 * v + 2], cs[3 * v],
                          cs[3 * v + 1], cs[3 * v + 2]);
  if (TQ)
    sym_apply_torque<Real, WALL>(c, k, t.z, f + 3 * K, own + 3 * K, acc[0], acc[1], acc[2], cs[0],
                                 cs[1], cs[2]);
}

// Tile pair (I, J), I <= J, of linear index Lp; its partials follow `pm` (one part, K
// vectors per slot), float32 in mixed precision.  Every lane of the workgroup must call this
// (it synchronises).
template <int K, bool TQ, bool WALL, typename Real, typename Part, typename Geom, typename Lds>
__device__ __forceinline__ void multi_tile_pair(const SymArgs &a, const Geom &g,
                                                const Real *__restrict__ src,
                                                const PairConsts<Real> &k,
                                                Part *__restrict__ partial, const PartMap &pm,
                                                int64_t Lp, int64_t I, int64_t J, Lds &L) {
  constexpr int R = src_rows<K, TQ>();
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
    for (int e = 0; e < R; ++e) L.f[e][tid] = src[e * a.stride + jb + tid];
  }
  __syncthreads();
  Real acc[3 * K];
#pragma unroll
  for (int e = 0; e < 3 * K; ++e) acc[e] = Real(0);
  if (I == J) {   // ordered pairs of the diagonal tile, self pair included
    for (int j = 0; j < cnt; ++j) {
      Real dx, dy;
      separation(t, L, j, dx, dy);
      SymCoef<Real> c;
      multi_coefficients<TQ, WALL>(dx, dy, t.z, L.z[j], k, c);
#pragma unroll
      for (int v = 0; v < K; ++v)
        sym_apply_one<Real, WALL>(c, L.f[3 * v][j], L.f[3 * v + 1][j], L.f[3 * v + 2][j],
                                  acc[3 * v], acc[3 * v + 1], acc[3 * v + 2]);
      if (TQ) {   // one direction: the target's own torque does not enter
        const Real tq[3] = {L.f[3 * K][j], L.f[3 * K + 1][j], L.f[3 * K + 2][j]};
        const Real none[3] = {Real(0), Real(0), Real(0)};
        Real px = Real(0), py = Real(0), pz = Real(0);
        sym_apply_torque<Real, WALL>(c, k, t.z, tq, none, acc[0], acc[1], acc[2], px, py, pz);
      }
    }
  } else {
    Real own[R];
#pragma unroll
    for (int e = 0; e < R; ++e) own[e] = on ? src[e * a.stride + i] : Real(0);
    for (int blk = 0; blk < cnt; blk += 64) {
      const int nb = min(64, cnt - blk);
      Real cs[3 * K];
#pragma unroll
      for (int e = 0; e < 3 * K; ++e) cs[e] = Real(0);
      if (nb == 64) {
        for (int step = 0; step < 64; ++step)
          multi_step<K, TQ, WALL>(L, blk + ((lane + step) & 63), true, t, own, k, acc, cs);
      } else {
        for (int step = 0; step < 64; ++step) {
          const int sl = (lane + step) & 63;
          multi_step<K, TQ, WALL>(L, blk + (sl < nb ? sl : 0), sl < nb, t, own, k, acc, cs);
        }
      }
      // after 64 rotations lane l holds the sums of source (l + 63) mod 64
      const int sl = (lane + 63) & 63;
#pragma unroll
      for (int e = 0; e < 3 * K; ++e) L.col[wave][e][sl] = cs[e];
      __syncthreads();
      for (int e0 = tid; e0 < 3 * K * 64; e0 += kBlock) {
        const int e = e0 / 64, s = e0 % 64;
        if (s < nb) {
          double sum = 0.0;
#pragma unroll
          for (int w = 0; w < kWaves; ++w) sum += double(L.col[w][e][s]);
          partial[part_elem(pm, Lp, 1, e / 3, e % 3, blk + s)] = Part(sum);
        }
      }
      __syncthreads();
    }
  }
  if (on)
#pragma unroll
    for (int e = 0; e < 3 * K; ++e)
      partial[part_elem(pm, Lp, 0, e / 3, e % 3, tid)] = Part(acc[e]);
}

// One workgroup per tile pair of the chunk [pm.L0, pm.L0 + gridDim.x).
template <int K, bool TQ, bool WALL>
__global__ __launch_bounds__(kBlock) void pair_kernel_mixed_multi(SymArgs a, PartMap pm, GeomF g,
                                                                  const float *__restrict__ src,
                                                                  PairConsts<float> k_arg,
                                                                  float *__restrict__ partial) {
  const PairConsts<float> k = vgpr_consts(k_arg);
  __shared__ MultiLdsF<K, TQ> L;
  int64_t I, J;
  const int64_t Lp = pm.L0 + int64_t(blockIdx.x);
  tri_decode(Lp, a.nt, I, J);
  multi_tile_pair<K, TQ, WALL>(a, g, src, k, partial, pm, Lp, I, J, L);
}

template <int K, bool TQ, bool WALL>
__global__ __launch_bounds__(kBlock) void pair_kernel_f64_multi(SymArgs a, PartMap pm, GeomD g,
                                                                const double *__restrict__ src,
                                                                PairConsts<double> k_arg,
                                                                double *__restrict__ partial) {
  const PairConsts<double> k = vgpr_consts(k_arg);
  __shared__ MultiLdsD<K, TQ> L;
  int64_t I, J;
  const int64_t Lp = pm.L0 + int64_t(blockIdx.x);
  tri_decode(Lp, a.nt, I, J);
  multi_tile_pair<K, TQ, WALL>(a, g, src, k, partial, pm, Lp, I, J, L);
}

// One thread per (vector slot, component, row): the chunk's partials added in a fixed order
// (chunk_row_sum), written to out.p[v] ([n][3]) on the first chunk and added on the others,
// scaled by H_i / (8 pi eta a) after the last.
template <int K, typename Part>
__global__ void reduce_multi(SymArgs a, PartMap pm, int64_t L1, int first, int last,
                             OutPtrs<K> out, const Part *__restrict__ partial,
                             const double *__restrict__ h, double scale) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = 3 * a.n;
  if (e >= K * per) return;
  const int v = int(e / per);
  const int64_t rem = e - int64_t(v) * per;
  const int d = int(rem / a.n);
  const int64_t r = rem - int64_t(d) * a.n;
  double *dst = out.p[v];
  if (!dst) return;
  double x = chunk_row_sum(partial, pm, a.nt, L1, r / kBlock, r % kBlock, v, d);
  if (!first) x += dst[3 * r + d];
  dst[3 * r + d] = last ? scale * h[r] * x : x;
}

// One product of K vectors: sources in.p[k] (slot 0 with torque `torque` when TQ), results to
// out.p[k].  The triangle of tile pairs is walked in chunks whose partials fit the context's
// limit,
// each chunk's pair kernel followed by its reduction into the results, so the workspace stays
// bounded whatever n.  The timing record spans the pair kernels of all chunks.
template <int K, bool TQ>
int multi_launch(rpb_ctx *ctx, const rpb_params *p, const Packed &g, SrcPtrs<K> in,
                 const double *torque, OutPtrs<K> out, hipStream_t stream) {
  const int64_t n = g.n;
  const bool f64 = g.precision == RPB_FP64;
  SymArgs a{n, kBlock, (n + kBlock - 1) / kBlock, n};
  const int64_t pairs = a.nt * (a.nt + 1) / 2;
  const size_t esz = f64 ? sizeof(double) : sizeof(float);
  const int64_t per_chunk = chunk_pairs(pairs, 1, K, kBlock, esz, ctx->chunk_bytes);
  int st;
  void *part = workspace(ctx, WS_PART, size_t(part_elems(per_chunk, 1, K, kBlock)) * esz, &st);
  if (!part) return st;
  void *src = workspace(ctx, WS_SRC, size_t(src_rows<K, TQ>()) * size_t(n) * esz, &st);
  if (!src) return st;
  const double *h = f64 ? geom_d(g).h : geom_f(g).h;
  int used = 0;
  for (int s = 0; s < K; ++s) used += in.p[s] != nullptr || (s == 0 && TQ);
  const double *tq = TQ ? torque : nullptr;
  if (f64)
    pack_multi<K, double><<<blocks_for(n, 256), 256, 0, stream>>>(n, in, h, tq, 1.0 / g.a,
                                                                 static_cast<double *>(src));
  else
    pack_multi<K, float><<<blocks_for(n, 256), 256, 0, stream>>>(n, in, h, tq, 1.0 / g.a,
                                                                static_cast<float *>(src));
  RPB_LAUNCHED(ctx);
  const double scale = 1.0 / (8.0 * M_PI * p->eta * p->a);
  hipEvent_t t0;
  RPB_TRY(timing_begin(ctx, stream, &t0));
  const bool wall = p->wall != 0;
  for (int64_t L0 = 0; L0 < pairs; L0 += per_chunk) {
    const int64_t L1 = std::min(pairs, L0 + per_chunk);
    const PartMap pm{L0, 1, kBlock, K};
    const unsigned grid = unsigned(L1 - L0);
    if (f64) {
      const auto k = make_pair_consts<double>();
      const auto *s = static_cast<const double *>(src);
      auto *pt = static_cast<double *>(part);
      if (wall)
        pair_kernel_f64_multi<K, TQ, true><<<grid, kBlock, 0, stream>>>(a, pm, geom_d(g), s, k, pt);
      else
        pair_kernel_f64_multi<K, TQ, false><<<grid, kBlock, 0, stream>>>(a, pm, geom_d(g), s, k,
                                                                        pt);
    } else {
      const auto k = make_pair_consts<float>();
      const auto *s = static_cast<const float *>(src);
      auto *pt = static_cast<float *>(part);
      if (wall)
        pair_kernel_mixed_multi<K, TQ, true><<<grid, kBlock, 0, stream>>>(a, pm, geom_f(g), s, k,
                                                                         pt);
      else
        pair_kernel_mixed_multi<K, TQ, false><<<grid, kBlock, 0, stream>>>(a, pm, geom_f(g), s, k,
                                                                          pt);
    }
    RPB_LAUNCHED(ctx);
    if (L1 == pairs)
      RPB_TRY(timing_end(ctx, stream, t0, double(n) * double(n) * used, 8 + (f64 ? 0 : 2)));
    const int first = L0 == 0, last = L1 == pairs;
    const unsigned rgrid = blocks_for(int64_t(K) * 3 * n, 256);
    if (f64)
      reduce_multi<K, double><<<rgrid, 256, 0, stream>>>(a, pm, L1, first, last, out,
                                                         static_cast<const double *>(part), h,
                                                         scale);
    else
      reduce_multi<K, float><<<rgrid, 256, 0, stream>>>(a, pm, L1, first, last, out,
                                                        static_cast<const float *>(part), h,
                                                        scale);
    RPB_LAUNCHED(ctx);
  }
  return RPB_OK;
}

// ---- batches of independent systems ------------------------------------------------------

struct MultiBatchArgs {
  const int64_t *offs;   // nsys + 1 sphere prefix sums
  const int64_t *cum;    // nsys + 1: first work item of each system, cum[nsys] = all items
  const int64_t *base;   // nsys + 1: first partial double of each system
  int nsys;
  int64_t n;             // total spheres (stride of the source arrays)
  int *counter;          // work counter (reset to 0 before the launch)
};

// Item and partial offsets of every system (one workgroup): system s has nt (nt + 1)/2 tile
// pairs of the upper triangle and part_elems(nt (nt + 1)/2, 1, K, kBlock) partials,
// nt = ceil(n_s / kBlock).
__global__ __launch_bounds__(kBlock) void multi_batch_setup(int nsys, int K,
                                                            const int64_t *__restrict__ offs,
                                                            int64_t *__restrict__ cum,
                                                            int64_t *__restrict__ base) {
  __shared__ int64_t pi[kBlock + 1], pe[kBlock + 1];
  const int tid = threadIdx.x;
  const int per = (nsys + kBlock - 1) / kBlock;
  const int s0 = min(nsys, tid * per), s1 = min(nsys, s0 + per);
  int64_t ci = 0, ce = 0;
  for (int s = s0; s < s1; ++s) {
    const int64_t nt = (offs[s + 1] - offs[s] + kBlock - 1) / kBlock;
    ci += nt * (nt + 1) / 2;
    ce += part_elems(nt * (nt + 1) / 2, 1, K, kBlock);
  }
  pi[tid] = ci;
  pe[tid] = ce;
  __syncthreads();
  if (tid == 0) {
    int64_t ri = 0, re = 0;
    for (int t = 0; t < kBlock; ++t) {
      const int64_t vi = pi[t], ve = pe[t];
      pi[t] = ri;
      pe[t] = re;
      ri += vi;
      re += ve;
    }
    pi[kBlock] = ri;
    pe[kBlock] = re;
  }
  __syncthreads();
  ci = pi[tid];
  ce = pe[tid];
  for (int s = s0; s < s1; ++s) {
    cum[s] = ci;
    base[s] = ce;
    const int64_t nt = (offs[s + 1] - offs[s] + kBlock - 1) / kBlock;
    ci += nt * (nt + 1) / 2;
    ce += part_elems(nt * (nt + 1) / 2, 1, K, kBlock);
  }
  if (tid == 0) {
    cum[nsys] = pi[kBlock];
    base[nsys] = pe[kBlock];
  }
}

// Next work item of the workgroup: (system, tile pair Lp = (I, J)), or false once the list is
// exhausted.  Every workgroup keeps pulling until the counter passes the item count, so every
// wave exits.
__device__ __forceinline__ bool next_multi_item(const MultiBatchArgs &b, int *slot, int &sys,
                                                int64_t &Lp, int64_t &I, int64_t &J) {
  __syncthreads();
  if (threadIdx.x == 0) slot[0] = atomicAdd(b.counter, 1);
  __syncthreads();
  const int64_t it = slot[0];
  if (it >= b.cum[b.nsys]) return false;
  int lo = 0, hi = b.nsys - 1;   // the last system with cum <= it (empty systems own no item)
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (b.cum[mid] <= it)
      lo = mid;
    else
      hi = mid - 1;
  }
  sys = lo;
  const int64_t nt = (b.offs[lo + 1] - b.offs[lo] + kBlock - 1) / kBlock;
  Lp = it - b.cum[lo];
  tri_decode(Lp, nt, I, J);
  return true;
}

__device__ __forceinline__ SymArgs multi_args_of(const MultiBatchArgs &b, int s) {
  const int64_t ns = b.offs[s + 1] - b.offs[s];
  return SymArgs{ns, kBlock, (ns + kBlock - 1) / kBlock, b.n};
}

template <int K, bool TQ, bool WALL>
__global__ __launch_bounds__(kBlock) void pair_kernel_mixed_multi_batched(
    MultiBatchArgs b, GeomF g, const float *__restrict__ src, PairConsts<float> k_arg,
    float *__restrict__ partial) {
  const PairConsts<float> k = vgpr_consts(k_arg);
  __shared__ MultiLdsF<K, TQ> L;
  __shared__ int slot[1];
  const PartMap pm{0, 1, kBlock, K};
  int s;
  int64_t Lp, I, J;
  while (next_multi_item(b, slot, s, Lp, I, J)) {
    const int64_t s0 = b.offs[s];
    multi_tile_pair<K, TQ, WALL>(multi_args_of(b, s), offset_geom(g, s0), src + s0, k,
                                 partial + b.base[s], pm, Lp, I, J, L);
  }
}

template <int K, bool TQ, bool WALL>
__global__ __launch_bounds__(kBlock) void pair_kernel_f64_multi_batched(
    MultiBatchArgs b, GeomD g, const double *__restrict__ src, PairConsts<double> k_arg,
    double *__restrict__ partial) {
  const PairConsts<double> k = vgpr_consts(k_arg);
  __shared__ MultiLdsD<K, TQ> L;
  __shared__ int slot[1];
  const PartMap pm{0, 1, kBlock, K};
  int s;
  int64_t Lp, I, J;
  while (next_multi_item(b, slot, s, Lp, I, J)) {
    const int64_t s0 = b.offs[s];
    multi_tile_pair<K, TQ, WALL>(multi_args_of(b, s), offset_geom(g, s0), src + s0, k,
                                 partial + b.base[s], pm, Lp, I, J, L);
  }
}

template <int K, typename Part>
__global__ void reduce_multi_batched(MultiBatchArgs b, const int *__restrict__ sys_of,
                                     OutPtrs<K> out, const Part *__restrict__ partial,
                                     const double *__restrict__ h, double scale) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = 3 * b.n;
  if (e >= K * per) return;
  const int v = int(e / per);
  const int64_t rem = e - int64_t(v) * per;
  const int d = int(rem / b.n);
  const int64_t r = rem - int64_t(d) * b.n;
  double *dst = out.p[v];
  if (!dst) return;
  const int s = sys_of[r];
  const SymArgs a = multi_args_of(b, s);
  const int64_t local = r - b.offs[s];
  const PartMap pm{0, 1, kBlock, K};
  dst[3 * r + d] = scale * h[r] *
                   chunk_row_sum(partial + b.base[s], pm, a.nt, a.nt * (a.nt + 1) / 2,
                                 local / kBlock, local % kBlock, v, d);
}

size_t multi_batch_partial_bytes(int K, const Batch &bt, size_t esz) {
  size_t bytes = 0;
  for (int s = 0; s < bt.nsys; ++s) {
    const int64_t nt = (bt.host_offs[s + 1] - bt.host_offs[s] + kBlock - 1) / kBlock;
    bytes += size_t(part_elems(nt * (nt + 1) / 2, 1, K, kBlock)) * esz;
  }
  return bytes;
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
  for (size_t g0 = 0; g0 < ids.size(); g0 += kMulti) {
    SrcPtrs<kMulti> in;
    OutPtrs<kMulti> out;
    for (int s = 0; s < kMulti; ++s) {
      const bool on = g0 + s < ids.size();
      const size_t off = on ? size_t(ids[g0 + s]) * 3 * n : 0;
      in.p[s] = on ? force + off : nullptr;
      out.p[s] = on ? vel + off : nullptr;
    }
    RPB_TRY((multi_launch<kMulti, false>(ctx, p, g, in, nullptr, out, stream)));
  }
  return RPB_OK;
}

bool matvec_first_supported(const rpb_params *p, int64_t n) { return p->lx <= 0.0 && n > 0; }

int matvec_first(rpb_ctx *ctx, const rpb_params *p, const Packed &g, const double *force,
                 const double *torque, const double *w, const double *w3, double *u_force,
                 double *u_w, double *u_w3, hipStream_t stream) {
  if (!matvec_first_supported(p, g.n))
    return fail(ctx, RPB_EINVAL, "joint product not available for this configuration");
  if (w3) {
    const SrcPtrs<3> in{{force, w, w3}};
    const OutPtrs<3> out{{u_force, u_w, u_w3}};
    if (torque) return multi_launch<3, true>(ctx, p, g, in, torque, out, stream);
    return multi_launch<3, false>(ctx, p, g, in, nullptr, out, stream);
  }
  const SrcPtrs<2> in{{force, w}};
  const OutPtrs<2> out{{u_force, u_w}};
  if (torque) return multi_launch<2, true>(ctx, p, g, in, torque, out, stream);
  return multi_launch<2, false>(ctx, p, g, in, nullptr, out, stream);
}

bool matvec_first_batched_supported(const rpb_params *p, const Batch &bt) {
  return p->lx <= 0.0 && bt.n > 0 && bt.nsys > 0 &&
         multi_batch_partial_bytes(2, bt, p->precision == RPB_FP64 ? sizeof(double)
                                                                   : sizeof(float)) <=
             kMaxMultiBatchBytes;
}

int matvec_first_batched(rpb_ctx *ctx, const rpb_params *p, const Batch &bt, const Packed &g,
                         const double *force, const double *torque, const double *w,
                         double *u_force, double *u_w, hipStream_t stream) {
  if (!matvec_first_batched_supported(p, bt))
    return fail(ctx, RPB_EINVAL, "joint batched product not available for this batch");
  constexpr int K = 2;
  const int64_t n = g.n;
  const bool f64 = g.precision == RPB_FP64;
  int st;
  const size_t meta_bytes = size_t(2 * (bt.nsys + 1)) * sizeof(int64_t);
  int64_t *meta = static_cast<int64_t *>(workspace(ctx, WS_MBATCH, meta_bytes, &st));
  if (!meta) return st;
  const size_t esz = f64 ? sizeof(double) : sizeof(float);
  void *part = workspace(ctx, WS_PART, std::max<size_t>(8, multi_batch_partial_bytes(K, bt, esz)),
                         &st);
  if (!part) return st;
  const bool tq = torque != nullptr;
  void *src = workspace(ctx, WS_SRC, size_t(3 * K + 3) * size_t(n) * esz, &st);
  if (!src) return st;
  char *small = static_cast<char *>(workspace(ctx, WS_SMALL, kSmallBytes, &st));
  if (!small) return st;
  int *counter = reinterpret_cast<int *>(small + kSmallWorkCounter);
  MultiBatchArgs args{bt.offs, meta, meta + bt.nsys + 1, bt.nsys, n, counter};
  multi_batch_setup<<<1, kBlock, 0, stream>>>(bt.nsys, K, bt.offs, meta, meta + bt.nsys + 1);
  RPB_LAUNCHED(ctx);
  const double *h = f64 ? geom_d(g).h : geom_f(g).h;
  const SrcPtrs<K> in{{force, w}};
  if (f64)
    pack_multi<K, double><<<blocks_for(n, 256), 256, 0, stream>>>(
        n, in, h, torque, 1.0 / g.a, static_cast<double *>(src));
  else
    pack_multi<K, float><<<blocks_for(n, 256), 256, 0, stream>>>(
        n, in, h, torque, 1.0 / g.a, static_cast<float *>(src));
  RPB_LAUNCHED(ctx);
  zero_counter<<<1, 1, 0, stream>>>(counter);
  RPB_LAUNCHED(ctx);
  const unsigned grid = unsigned(std::max(1, bt.wgs));
  hipEvent_t t0;
  RPB_TRY(timing_begin(ctx, stream, &t0));
  const bool wall = p->wall != 0;
  auto launch = [&](auto TQ) {
    constexpr bool kTQ = decltype(TQ)::value;
    if (f64) {
      const auto k = make_pair_consts<double>();
      const auto *s = static_cast<const double *>(src);
      auto *pt = static_cast<double *>(part);
      if (wall)
        pair_kernel_f64_multi_batched<K, kTQ, true><<<grid, kBlock, 0, stream>>>(args, geom_d(g),
                                                                                 s, k, pt);
      else
        pair_kernel_f64_multi_batched<K, kTQ, false><<<grid, kBlock, 0, stream>>>(
            args, geom_d(g), s, k, pt);
    } else {
      const auto k = make_pair_consts<float>();
      const auto *s = static_cast<const float *>(src);
      auto *pt = static_cast<float *>(part);
      if (wall)
        pair_kernel_mixed_multi_batched<K, kTQ, true><<<grid, kBlock, 0, stream>>>(
            args, geom_f(g), s, k, pt);
      else
        pair_kernel_mixed_multi_batched<K, kTQ, false><<<grid, kBlock, 0, stream>>>(
            args, geom_f(g), s, k, pt);
    }
  };
  if (tq)
    launch(std::true_type{});
  else
    launch(std::false_type{});
  RPB_LAUNCHED(ctx);
  double pairs = 0.0;
  for (int q = 0; q < bt.nsys; ++q) {
    const double ns = double(bt.host_offs[q + 1] - bt.host_offs[q]);
    pairs += ns * ns;
  }
  RPB_TRY(timing_end(ctx, stream, t0, K * pairs, 8 + (f64 ? 0 : 2)));
  const double scale = 1.0 / (8.0 * M_PI * p->eta * p->a);
  const OutPtrs<K> out{{u_force, u_w}};
  if (f64)
    reduce_multi_batched<K, double><<<blocks_for(int64_t(K) * 3 * n, 256), 256, 0, stream>>>(
        args, bt.sys_of, out, static_cast<const double *>(part), h, scale);
  else
    reduce_multi_batched<K, float><<<blocks_for(int64_t(K) * 3 * n, 256), 256, 0, stream>>>(
        args, bt.sys_of, out, static_cast<const float *>(part), h, scale);
  RPB_LAUNCHED(ctx);
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
