// Device-side pieces shared by the pair kernels (matvec.hip, multi.hip): packed-geometry views,
// the compensated float32 sum, and the tiling of the symmetric tile-pair kernels.
#pragma once

#include <cstdint>

#include "pair_tensor.h"
#include "rpb_internal.h"

namespace rpb {

namespace {

constexpr int kBlock = 256;   // lanes per workgroup = targets per tile row = sources per LDS tile

struct GeomD {         // float64 geometry: x, y, z~ and H, n each
  const double *x, *y, *z, *h;
};
struct GeomF {         // mixed geometry: float32 hi/lo x, y, float32 z~, float64 H
  const float *xh, *xl, *yh, *yl, *z;
  const double *h;
};

inline GeomD geom_d(const Packed &g) {
  const double *b = static_cast<const double *>(g.geom);
  return {b, b + g.n, b + 2 * g.n, b + 3 * g.n};
}
inline GeomF geom_f(const Packed &g) {
  const double *h = static_cast<const double *>(g.geom);
  const float *f = reinterpret_cast<const float *>(h + g.n);
  return {f, f + g.n, f + 2 * g.n, f + 3 * g.n, f + 4 * g.n, h};
}
inline size_t geom_bytes(int64_t n, int precision) {
  return precision == RPB_FP64 ? size_t(4 * n) * sizeof(double)
                               : size_t(n) * sizeof(double) + size_t(5 * n) * sizeof(float);
}

// The geometry of a batch's system starting at sphere s0.
inline __device__ GeomF offset_geom(const GeomF &g, int64_t s0) {
  return {g.xh + s0, g.xl + s0, g.yh + s0, g.yl + s0, g.z + s0, g.h + s0};
}
inline __device__ GeomD offset_geom(const GeomD &g, int64_t s0) {
  return {g.x + s0, g.y + s0, g.z + s0, g.h + s0};
}

__device__ __forceinline__ void kahan_add(float &s, float &c, float v) {
  const float y = v - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}

struct SymArgs {
  int64_t n;           // spheres of the system
  int64_t ts;          // tile size (kBlock * TPT)
  int64_t nt;          // tiles
  int64_t stride;      // stride of the source component arrays (all systems' spheres)
  int64_t nsplit = 1;  // workgroups per tile pair, each taking one part of the source tile
  const int *skip = nullptr;   // optional device flag: the launch does nothing while it is nonzero
};

// v from lane (l + 1) mod 64 (DPP wave_rol:1).  Every lane has a source lane, so the "old"
// operand is never used; passing v itself lets the move be done in place.
__device__ __forceinline__ float wave_rol1(float v) {
  const int b = __float_as_int(v);
  return __int_as_float(__builtin_amdgcn_update_dpp(b, b, 0x134, 0xf, 0xf, false));
}
__device__ __forceinline__ double wave_rol1(double v) {
  const long long b = __double_as_longlong(v);
  const int l = int(b & 0xffffffffll), h = int(b >> 32);
  const int lo = __builtin_amdgcn_update_dpp(l, l, 0x134, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(h, h, 0x134, 0xf, 0xf, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<long long>(static_cast<unsigned>(lo)));
}

constexpr int kWaves = kBlock / 64;

// Tile pairs (I, J), I <= J, of the upper triangle in row-major order: pair (I, J) has linear
// index L = tri_start(I) + J - I, row I holding nt - I pairs.
__host__ __device__ __forceinline__ int64_t tri_start(int64_t r, int64_t nt) {
  return r * nt - r * (r - 1) / 2;
}

// (I, J) of linear index L.  Workgroups walk the triangle row by row.
__device__ __forceinline__ void tri_decode(int64_t L, int64_t nt, int64_t &I, int64_t &J) {
  const double b = double(2 * nt + 1);
  int64_t i = int64_t((b - sqrt(b * b - 8.0 * double(L))) * 0.5);
  if (i < 0) i = 0;
  if (i > nt - 1) i = nt - 1;
  while (i > 0 && tri_start(i, nt) > L) --i;
  while (i + 1 < nt && tri_start(i + 1, nt) <= L) ++i;
  I = i;
  J = i + (L - tri_start(i, nt));
}

// Partial sums of the symmetric tile-pair kernels.  One launch covers the tile pairs of linear
// index L in [L0, L1) (a chunk of the triangle; the whole triangle when it fits the workspace
// limit).  Pair q = L - L0 owns nsplit + 1 slots: slot q (nsplit + 1) + h holds the sums for
// the rows of tile I over source part h of tile J (h < nsplit), slot q (nsplit + 1) + nsplit
// the sums for the rows of tile J over tile I (I < J only; each part writes its own rows of
// it).  A slot holds V vectors x 3 components x ts rows.
struct PartMap {
  int64_t L0;       // first pair of the chunk
  int64_t nsplit;   // source parts per tile pair
  int64_t ts;       // rows per tile
  int V;            // vectors per slot
};

__host__ __device__ __forceinline__ int64_t part_elem(const PartMap &m, int64_t L, int64_t sub,
                                                      int v, int comp, int64_t local) {
  return ((((L - m.L0) * (m.nsplit + 1) + sub) * m.V + v) * 3 + comp) * m.ts + local;
}

// Elements of the partial buffer of pairs [L0, L1).
__host__ __device__ __forceinline__ int64_t part_elems(int64_t pairs, int64_t nsplit, int V,
                                                       int64_t ts) {
  return pairs * (nsplit + 1) * V * 3 * ts;
}

// Sum, in a fixed order, of every partial of row `local` of tile T (component c, vector v)
// that the pairs [L0, L1) wrote: first the column slots of pairs (I, T), I < T, in increasing I,
// then the row slots of pairs (T, J), J >= T, in increasing J (the parts of each pair summed
// in four interleaved sums, h mod 4, combined in a fixed order).  Four
// running sums keep several loads in flight.  L(I, T) increases with I, so the pairs (I, T) of
// the chunk form one range of I, found by bisection.
template <typename Part>
__device__ __forceinline__ double chunk_row_sum(const Part *__restrict__ p, const PartMap &m,
                                                int64_t nt, int64_t L1, int64_t T, int64_t local,
                                                int v, int c) {
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int k = 0;
  auto Lcol = [&](int64_t I) { return tri_start(I, nt) + T - I; };
  int64_t lo = 0, hi = T;
  while (lo < hi) {   // first I with L(I, T) >= L0
    const int64_t mid = (lo + hi) / 2;
    if (Lcol(mid) >= m.L0)
      hi = mid;
    else
      lo = mid + 1;
  }
  const int64_t i0 = lo;
  hi = T;
  while (lo < hi) {   // first I with L(I, T) >= L1
    const int64_t mid = (lo + hi) / 2;
    if (Lcol(mid) >= L1)
      hi = mid;
    else
      lo = mid + 1;
  }
  for (int64_t I = i0; I < lo; ++I)
    s[k++ & 3] += double(p[part_elem(m, Lcol(I), m.nsplit, v, c, local)]);
  const int64_t st = tri_start(T, nt);
  const int64_t j0 = T + (m.L0 > st ? m.L0 - st : 0);
  const int64_t j1 = T + (L1 - st < nt - T ? (L1 > st ? L1 - st : 0) : nt - T);
  for (int64_t J = j0; J < j1; ++J) {
    const int64_t L = st + J - T;
    // the parts of the pair in four running sums (h mod 4), so that many parts (small systems
    // split into up to 128) keep several loads in flight
    double x[4] = {double(p[part_elem(m, L, 0, v, c, local)]), 0.0, 0.0, 0.0};
    for (int64_t h = 1; h < m.nsplit; ++h) x[h & 3] += double(p[part_elem(m, L, h, v, c, local)]);
    s[k++ & 3] += (x[0] + x[1]) + (x[2] + x[3]);
  }
  return (s[0] + s[1]) + (s[2] + s[3]);
}

// The same partials as chunk_row_sum for one vector, shared by G threads: the slots, in the
// order of chunk_row_sum (column slots of pairs (I, T) in increasing I, then the parts h of the
// row slots of pairs (T, J) in increasing J and h), are dealt to the G threads in turn; thread g
// adds slots g + (4 j + q) G into running sum q, four loads in flight, and returns
// (s_0 + s_1) + (s_2 + s_3).  The caller adds the G results in a fixed order.
template <typename Part>
__device__ __forceinline__ double chunk_row_sum_dealt(const Part *__restrict__ p,
                                                      const PartMap &m, int64_t nt, int64_t L1,
                                                      int64_t T, int64_t local, int c, int g,
                                                      int G) {
  auto Lcol = [&](int64_t I) { return tri_start(I, nt) + T - I; };
  int64_t lo = 0, hi = T;
  while (lo < hi) {   // first I with L(I, T) >= L0
    const int64_t mid = (lo + hi) / 2;
    if (Lcol(mid) >= m.L0)
      hi = mid;
    else
      lo = mid + 1;
  }
  const int64_t i0 = lo;
  hi = T;
  while (lo < hi) {   // first I with L(I, T) >= L1
    const int64_t mid = (lo + hi) / 2;
    if (Lcol(mid) >= L1)
      hi = mid;
    else
      lo = mid + 1;
  }
  const int ncol = int(lo - i0);
  const int64_t st = tri_start(T, nt);
  const int64_t j0 = T + (m.L0 > st ? m.L0 - st : 0);
  const int64_t j1 = T + (L1 - st < nt - T ? (L1 > st ? L1 - st : 0) : nt - T);
  const int ns = int(m.nsplit);
  const int nslots = ncol + int(j1 - j0) * ns;
  auto slot = [&](int q) -> double {   // value of slot q < nslots
    if (q < ncol) return double(p[part_elem(m, Lcol(i0 + q), m.nsplit, 0, c, local)]);
    const int t = q - ncol;
    const int64_t J = j0 + t / ns;
    return double(p[part_elem(m, st + J - T, t % ns, 0, c, local)]);
  };
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int q = g; q < nslots; q += 4 * G) {
    double x[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) x[r] = q + r * G < nslots ? slot(q + r * G) : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) s[r] += x[r];
  }
  return (s[0] + s[1]) + (s[2] + s[3]);
}

// Chunks of the triangle: at most `limit` bytes of partials per launch (the context's chunk
// limit, kMaxChunkBytes unless overridden), equal numbers of pairs per chunk.
inline int64_t chunk_pairs(int64_t pairs, int64_t nsplit, int V, int64_t ts, size_t esz,
                           size_t limit) {
  const size_t per = size_t(part_elems(1, nsplit, V, ts)) * esz;
  int64_t fit = int64_t(limit / per);
  if (fit < 1) fit = 1;
  if (fit > 0x7fffffffll / nsplit) fit = 0x7fffffffll / nsplit;
  const int64_t nchunks = (pairs + fit - 1) / fit;
  return (pairs + nchunks - 1) / nchunks;   // equal chunks
}

inline unsigned blocks_for(int64_t n, int threads) {
  return unsigned((n + threads - 1) / threads);
}

}  // namespace

}  // namespace rpb
