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

// slot (T, P, h) of the symmetric partial array:
// partial[(((T * nt + P) * nsplit + h) * 3 + comp) * ts + local].  Tile T's rows get the sums
// over source part h of tile P in slot (T, P, h) when T <= P, and the column sums of the
// tile pair (P, T) in slot (T, P, 0) when T > P.
__device__ __forceinline__ int64_t sym_slot(const SymArgs &a, int64_t T, int64_t P, int comp,
                                            int64_t local, int64_t h = 0) {
  return (((T * a.nt + P) * a.nsplit + h) * 3 + comp) * a.ts + local;
}

constexpr int kWaves = kBlock / 64;

// Tile pair (I, J), I <= J, of linear index L = I nt - I (I - 1) / 2 + (J - I): row I of the
// upper triangle holds nt - I pairs.  Workgroups walk the triangle row by row.
__device__ __forceinline__ void tri_decode(int64_t L, int64_t nt, int64_t &I, int64_t &J) {
  const double b = double(2 * nt + 1);
  int64_t i = int64_t((b - sqrt(b * b - 8.0 * double(L))) * 0.5);
  auto start = [nt](int64_t r) { return r * nt - r * (r - 1) / 2; };
  if (i < 0) i = 0;
  if (i > nt - 1) i = nt - 1;
  while (i > 0 && start(i) > L) --i;
  while (i + 1 < nt && start(i + 1) <= L) ++i;
  I = i;
  J = i + (L - start(i));
}

inline unsigned blocks_for(int64_t n, int threads) {
  return unsigned((n + threads - 1) / threads);
}

}  // namespace

}  // namespace rpb
