// Matrix-free product U = M F + M_C T of the regularised Rotne-Prager-Blake mobility.
//
// Direct summation over all pairs (paper, Sec. II.B): the pair tensor is evaluated on the fly
// (pair_tensor.h) and never stored, so the kernels are bound by the vector ALUs, not by HBM.
// Layout:
//   pack_geometry   O(N)   AoS float64 positions -> SoA lengths in units of a, clamped heights,
//                          weights H0(z/a) (App. A, eq. effMob); mixed precision splits x, y
//                          into float32 hi + lo so that near-pair separations keep ~1e-7
//                          accuracy far from the origin.
//   pack_vectors    O(N)   AoS float64 force/torque -> SoA H-weighted source vectors (torques
//                          divided by a).
//   pair kernels    O(N^2) * whole system: the symmetric tile-pair kernel, one evaluation
//                            per unordered pair applied in both directions (M_ji = M_ij^T);
//                          * row ranges: a workgroup owns a tile of targets (kBlock lanes x
//                            TPT targets per lane) and streams a chunk of sources through LDS;
//                          * batched systems: persistent workgroups pull (system, tile pair)
//                            or (system, target tile, source chunk) items, largest first.
//                          Float64 sums, or float32 sums per LDS tile added with Kahan
//                          compensation.
//   reduce_partials O(N S) fixed-order sum of the partials, times H_i / (8 pi eta a).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <type_traits>

#include "pair_common.h"

namespace rpb {

namespace {

// Positions in units of a.  With a wall: z~ = max(z, a) and H = clamp(z/a, 0, 1) (App. A); in
// free space: z~ = z, H = 1.
__global__ void pack_geometry_f64(int64_t n, const double *__restrict__ pos, double a, int wall,
                                  double *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double z = pos[3 * i + 2] / a;
  out[i] = pos[3 * i] / a;
  out[n + i] = pos[3 * i + 1] / a;
  out[2 * n + i] = wall ? fmax(z, 1.0) : z;
  out[3 * n + i] = wall ? fmin(fmax(z, 0.0), 1.0) : 1.0;
}

__global__ void pack_geometry_mixed(int64_t n, const double *__restrict__ pos, double a,
                                    int wall, double *__restrict__ hout, float *__restrict__ f) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = pos[3 * i] / a, y = pos[3 * i + 1] / a, z = pos[3 * i + 2] / a;
  const float xh = float(x), yh = float(y);
  f[i] = xh;
  f[n + i] = float(x - double(xh));
  f[2 * n + i] = yh;
  f[3 * n + i] = float(y - double(yh));
  f[4 * n + i] = float(wall ? fmax(z, 1.0) : z);
  hout[i] = wall ? fmin(fmax(z, 0.0), 1.0) : 1.0;
}

// Source vectors, H-weighted, structure of arrays: [fx | fy | fz | tx | ty | tz] (n each); the
// torques divided by a (lengths in units of a).
template <typename Real>
__global__ void pack_vectors(int64_t n, const double *__restrict__ h,
                             const double *__restrict__ force, const double *__restrict__ torque,
                             double inv_a, Real *__restrict__ out, const int *__restrict__ skip) {
  if (skip && *skip) return;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double w = h[i];
  for (int c = 0; c < 3; ++c) {
    out[c * n + i] = force ? Real(w * force[3 * i + c]) : Real(0);
    if (torque) out[(3 + c) * n + i] = Real(w * inv_a * torque[3 * i + c]);
  }
}


// ---- workgroup-level building blocks shared by the single and batched kernels ---------------

template <bool TORQUE>
struct LdsD {
  double x[kBlock], y[kBlock], z[kBlock];
  double f[3][kBlock];
  double t[TORQUE ? 3 : 1][kBlock];
};
template <bool TORQUE>
struct LdsF {
  float xh[kBlock], xl[kBlock], yh[kBlock], yl[kBlock], z[kBlock];
  float f[3][kBlock];
  float t[TORQUE ? 3 : 1][kBlock];
};

template <int TPT>
struct TargetsD {
  double x[TPT], y[TPT], z[TPT];
  double u[TPT][3];
};
template <int TPT>
struct TargetsF {
  float xh[TPT], xl[TPT], yh[TPT], yl[TPT], z[TPT];
  float s[TPT][3], c[TPT][3];     // Kahan sum and compensation
};

// Load the lane's targets: rows first + q * kBlock + tid for q < TPT (row `safe` when out of
// range, which keeps every load in bounds; such targets are never stored).
template <int TPT>
__device__ __forceinline__ void load_targets(const GeomD &g, int64_t first, int64_t end,
                                             int64_t safe, TargetsD<TPT> &T) {
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int64_t r = first + q * kBlock + threadIdx.x;
    const int64_t i = r < end ? r : safe;
    T.x[q] = g.x[i];
    T.y[q] = g.y[i];
    T.z[q] = g.z[i];
    T.u[q][0] = T.u[q][1] = T.u[q][2] = 0.0;
  }
}
template <int TPT>
__device__ __forceinline__ void load_targets(const GeomF &g, int64_t first, int64_t end,
                                             int64_t safe, TargetsF<TPT> &T) {
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int64_t r = first + q * kBlock + threadIdx.x;
    const int64_t i = r < end ? r : safe;
    T.xh[q] = g.xh[i];
    T.xl[q] = g.xl[i];
    T.yh[q] = g.yh[i];
    T.yl[q] = g.yl[i];
    T.z[q] = g.z[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) T.s[q][d] = T.c[q][d] = 0.f;
  }
}

// Accumulate sources [jb, je) into the lane's targets.  `n` is the stride of the source
// arrays.  Every lane of the workgroup must call this (it synchronises).
template <bool TORQUE, int TPT, bool WALL, bool PERIODIC>
__device__ __forceinline__ void sources_f64(const GeomD &g, const double *__restrict__ src,
                                            int64_t n, int64_t jb, int64_t je,
                                            const PairConsts<double> &k, LdsD<TORQUE> &L,
                                            TargetsD<TPT> &T) {
  const int tid = threadIdx.x;
  for (int64_t t0 = jb; t0 < je; t0 += kBlock) {
    const int cnt = int(min<int64_t>(kBlock, je - t0));
    __syncthreads();
    if (tid < cnt) {
      const int64_t j = t0 + tid;
      L.x[tid] = g.x[j];
      L.y[tid] = g.y[j];
      L.z[tid] = g.z[j];
      L.f[0][tid] = src[j];
      L.f[1][tid] = src[n + j];
      L.f[2][tid] = src[2 * n + j];
      if (TORQUE) {
        L.t[0][tid] = src[3 * n + j];
        L.t[1][tid] = src[4 * n + j];
        L.t[2][tid] = src[5 * n + j];
      }
    }
    __syncthreads();
#pragma unroll 2
    for (int j = 0; j < cnt; ++j) {
      const double xj = L.x[j], yj = L.y[j], zj = L.z[j];
      const double fx = L.f[0][j], fy = L.f[1][j], fz = L.f[2][j];
      const double tx = TORQUE ? L.t[0][j] : 0.0, ty = TORQUE ? L.t[1][j] : 0.0,
                   tz = TORQUE ? L.t[2][j] : 0.0;
      // pairs closer than 2a (rare) and the self pair take the complete form
#pragma unroll
      for (int q = 0; q < TPT; ++q) {
        for_images<PERIODIC>(T.x[q] - xj, T.y[q] - yj, k, [&](double dx, double dy) {
          const double dz = T.z[q] - zj;
          if (dx * dx + dy * dy + dz * dz < kFourA2)
            pair_velocity<double, TORQUE, false, WALL>(dx, dy, T.z[q], zj, fx, fy, fz, tx, ty,
                                                       tz, k, T.u[q][0], T.u[q][1], T.u[q][2]);
          else
            pair_velocity<double, TORQUE, true, WALL>(dx, dy, T.z[q], zj, fx, fy, fz, tx, ty,
                                                      tz, k, T.u[q][0], T.u[q][1], T.u[q][2]);
        });
      }
    }
  }
}

template <bool TORQUE, int TPT, bool WALL, bool PERIODIC>
__device__ __forceinline__ void sources_mixed(const GeomF &g, const float *__restrict__ src,
                                              int64_t n, int64_t jb, int64_t je,
                                              const PairConsts<float> &k, LdsF<TORQUE> &L,
                                              TargetsF<TPT> &T) {
  const int tid = threadIdx.x;
  for (int64_t t0 = jb; t0 < je; t0 += kBlock) {
    const int cnt = int(min<int64_t>(kBlock, je - t0));
    __syncthreads();
    if (tid < cnt) {
      const int64_t j = t0 + tid;
      L.xh[tid] = g.xh[j];
      L.xl[tid] = g.xl[j];
      L.yh[tid] = g.yh[j];
      L.yl[tid] = g.yl[j];
      L.z[tid] = g.z[j];
      L.f[0][tid] = src[j];
      L.f[1][tid] = src[n + j];
      L.f[2][tid] = src[2 * n + j];
      if (TORQUE) {
        L.t[0][tid] = src[3 * n + j];
        L.t[1][tid] = src[4 * n + j];
        L.t[2][tid] = src[5 * n + j];
      }
    }
    __syncthreads();
    float a[TPT][3];
#pragma unroll
    for (int q = 0; q < TPT; ++q) a[q][0] = a[q][1] = a[q][2] = 0.f;
#pragma unroll 2
    for (int j = 0; j < cnt; ++j) {
      const float xjh = L.xh[j], xjl = L.xl[j], yjh = L.yh[j], yjl = L.yl[j], zj = L.z[j];
      const float fx = L.f[0][j], fy = L.f[1][j], fz = L.f[2][j];
      const float tx = TORQUE ? L.t[0][j] : 0.f, ty = TORQUE ? L.t[1][j] : 0.f,
                  tz = TORQUE ? L.t[2][j] : 0.f;
      // pairs closer than 2a (rare) and the self pair take the complete form
#pragma unroll
      for (int q = 0; q < TPT; ++q) {
        const float dx0 = (T.xh[q] - xjh) + (T.xl[q] - xjl);
        const float dy0 = (T.yh[q] - yjh) + (T.yl[q] - yjl);
        for_images<PERIODIC>(dx0, dy0, k, [&](float dx, float dy) {
          const float dz = T.z[q] - zj;
          if (dx * dx + dy * dy + dz * dz < float(kFourA2))
            pair_velocity<float, TORQUE, false, WALL>(dx, dy, T.z[q], zj, fx, fy, fz, tx, ty, tz,
                                                      k, a[q][0], a[q][1], a[q][2]);
          else
            pair_velocity<float, TORQUE, true, WALL>(dx, dy, T.z[q], zj, fx, fy, fz, tx, ty, tz,
                                                     k, a[q][0], a[q][1], a[q][2]);
        });
      }
    }
#pragma unroll
    for (int q = 0; q < TPT; ++q)
#pragma unroll
      for (int d = 0; d < 3; ++d) kahan_add(T.s[q][d], T.c[q][d], a[q][d]);
  }
}

// partial[(chunk * 3 + comp) * stride + (row - base_row)] for the lane's targets below `end`
template <int TPT>
__device__ __forceinline__ void store_partial(const TargetsD<TPT> &T, int64_t first, int64_t end,
                                              int64_t chunk, int64_t stride, int64_t base_row,
                                              double *__restrict__ partial) {
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int64_t r = first + q * kBlock + threadIdx.x;
    if (r < end) {
      const int64_t o = chunk * 3 * stride + (r - base_row);
      partial[o] = T.u[q][0];
      partial[o + stride] = T.u[q][1];
      partial[o + 2 * stride] = T.u[q][2];
    }
  }
}
template <int TPT>
__device__ __forceinline__ void store_partial(const TargetsF<TPT> &T, int64_t first, int64_t end,
                                              int64_t chunk, int64_t stride, int64_t base_row,
                                              double *__restrict__ partial) {
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int64_t r = first + q * kBlock + threadIdx.x;
    if (r < end) {
      const int64_t o = chunk * 3 * stride + (r - base_row);
      partial[o] = double(T.s[q][0]) - double(T.c[q][0]);
      partial[o + stride] = double(T.s[q][1]) - double(T.c[q][1]);
      partial[o + 2 * stride] = double(T.s[q][2]) - double(T.c[q][2]);
    }
  }
}

// ---- single system: grid (target tile, source chunk) -----------------------------------------

struct PairArgs {
  int64_t n;        // sources (and geometry size)
  int64_t row0;     // first target
  int64_t nrows;    // number of targets
  int64_t chunk;    // sources per workgroup (multiple of kBlock)
  const int *skip;  // optional device flag: the launch does nothing while it is nonzero
};

template <bool TORQUE, int TPT, bool WALL, bool PERIODIC>
__global__ __launch_bounds__(kBlock) void pair_kernel_f64(PairArgs args, GeomD g,
                                                          const double *__restrict__ src,
                                                          PairConsts<double> k_arg,
                                                          double *__restrict__ partial) {
  const PairConsts<double> k = vgpr_consts(k_arg);
  if (args.skip && *args.skip) return;
  __shared__ LdsD<TORQUE> L;
  TargetsD<TPT> T;
  const int64_t first = args.row0 + int64_t(blockIdx.x) * (kBlock * TPT);
  const int64_t end = args.row0 + args.nrows;
  load_targets<TPT>(g, first, end, args.row0, T);
  const int64_t jb = int64_t(blockIdx.y) * args.chunk;
  sources_f64<TORQUE, TPT, WALL, PERIODIC>(g, src, args.n, jb, min(args.n, jb + args.chunk), k,
                                           L, T);
  store_partial<TPT>(T, first, end, blockIdx.y, args.nrows, args.row0, partial);
}

template <bool TORQUE, int TPT, bool WALL, bool PERIODIC>
__global__ __launch_bounds__(kBlock) void pair_kernel_mixed(PairArgs args, GeomF g,
                                                            const float *__restrict__ src,
                                                            PairConsts<float> k_arg,
                                                            double *__restrict__ partial) {
  const PairConsts<float> k = vgpr_consts(k_arg);
  if (args.skip && *args.skip) return;
  __shared__ LdsF<TORQUE> L;
  TargetsF<TPT> T;
  const int64_t first = args.row0 + int64_t(blockIdx.x) * (kBlock * TPT);
  const int64_t end = args.row0 + args.nrows;
  load_targets<TPT>(g, first, end, args.row0, T);
  const int64_t jb = int64_t(blockIdx.y) * args.chunk;
  sources_mixed<TORQUE, TPT, WALL, PERIODIC>(g, src, args.n, jb, min(args.n, jb + args.chunk), k,
                                             L, T);
  store_partial<TPT>(T, first, end, blockIdx.y, args.nrows, args.row0, partial);
}

__global__ void reduce_partials(int64_t nrows, int nchunks, const double *__restrict__ partial,
                                const double *__restrict__ h, double scale,
                                double *__restrict__ vel, const int *__restrict__ skip) {
  if (skip && *skip) return;
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const double w = scale * h[r];
  for (int c = 0; c < 3; ++c) {
    double s = 0.0;
    for (int q = 0; q < nchunks; ++q) s += partial[(int64_t(q) * 3 + c) * nrows + r];
    vel[3 * r + c] = w * s;
  }
}

// ---- single system, force-only sources: one evaluation per unordered pair ------------------
//
// The mobility matrix is symmetric, so a workgroup owning target tile I and source tile J > I
// evaluates each pair (i, j) once (pair_velocity_sym) and produces both M_ij F_j (summed per
// target in registers) and M_ij^T F_i = M_ji F_i (summed per source).  Within a wavefront the
// sources are taken in blocks of 64 on a rotating schedule: at step k lane l works on source
// (l + k) mod 64, and the per-source sums travel one lane down per step (DPP wave_rol:1), so
// after 64 steps lane l holds the complete sum over the wavefront's targets for source
// (l + 63) mod 64 without any cross-lane reduction.  The wavefronts' sums are added in LDS in
// a fixed order.  Tile I gets slot (I, J) and tile J gets slot (J, I) of the partial array;
// diagonal tiles are evaluated as ordered pairs into slot (I, I).  Every target thus receives
// exactly nt partials, summed in slot order.

// One rotation step: every lane passes its per-source sums cs one lane down, then evaluates
// its targets against source j (weighted force zero when !valid), adding M_ij F_j into acc and
// M_ij^T F_i into cs.  Pairs at least 2a apart use the far-field form alone; closer pairs (rare
// in a suspension) the complete form, so each pair's value depends on its own geometry only.
template <int TPT, bool TORQUE, bool WALL, bool PERIODIC>
__device__ __forceinline__ void sym_step(const LdsF<TORQUE> &L, int j, bool valid,
                                         const TargetsF<TPT> &T, const float (&own)[TPT][6],
                                         const PairConsts<float> &k, float (&acc)[TPT][3],
                                         float (&cs)[3]) {
  const float xjh = L.xh[j], xjl = L.xl[j], yjh = L.yh[j], yjl = L.yl[j], zj = L.z[j];
  const float fx = valid ? L.f[0][j] : 0.f, fy = valid ? L.f[1][j] : 0.f,
              fz = valid ? L.f[2][j] : 0.f;
  float tq[3] = {0.f, 0.f, 0.f};
  if (TORQUE) {
#pragma unroll
    for (int c = 0; c < 3; ++c) tq[c] = valid ? L.t[c][j] : 0.f;
  }
  // the sums start at zero, so the first step rotates zeros
#pragma unroll
  for (int c = 0; c < 3; ++c) cs[c] = wave_rol1(cs[c]);
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const float dx0 = (T.xh[q] - xjh) + (T.xl[q] - xjl);
    const float dy0 = (T.yh[q] - yjh) + (T.yl[q] - yjl);
    for_images<PERIODIC>(dx0, dy0, k, [&](float dx, float dy) {
      const float dz = T.z[q] - zj;
      if (dx * dx + dy * dy + dz * dz < float(kFourA2))
        pair_velocity_sym<float, false, TORQUE, WALL>(dx, dy, T.z[q], zj, fx, fy, fz, own[q][0],
                                                      own[q][1], own[q][2], k, acc[q][0],
                                                      acc[q][1], acc[q][2], cs[0], cs[1], cs[2],
                                                      tq, own[q] + 3);
      else
        pair_velocity_sym<float, true, TORQUE, WALL>(dx, dy, T.z[q], zj, fx, fy, fz, own[q][0],
                                                     own[q][1], own[q][2], k, acc[q][0],
                                                     acc[q][1], acc[q][2], cs[0], cs[1], cs[2], tq,
                                                     own[q] + 3);
    });
  }
}

template <int TPT, bool TORQUE, bool WALL, bool PERIODIC>
__device__ __forceinline__ void sym_step(const LdsD<TORQUE> &L, int j, bool valid,
                                         const TargetsD<TPT> &T, const double (&own)[TPT][6],
                                         const PairConsts<double> &k, double (&acc)[TPT][3],
                                         double (&cs)[3]) {
  const double xj = L.x[j], yj = L.y[j], zj = L.z[j];
  const double fx = valid ? L.f[0][j] : 0.0, fy = valid ? L.f[1][j] : 0.0,
               fz = valid ? L.f[2][j] : 0.0;
  double tq[3] = {0.0, 0.0, 0.0};
  if (TORQUE) {
#pragma unroll
    for (int c = 0; c < 3; ++c) tq[c] = valid ? L.t[c][j] : 0.0;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) cs[c] = wave_rol1(cs[c]);
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    for_images<PERIODIC>(T.x[q] - xj, T.y[q] - yj, k, [&](double dx, double dy) {
      const double dz = T.z[q] - zj;
      if (dx * dx + dy * dy + dz * dz < kFourA2)
        pair_velocity_sym<double, false, TORQUE, WALL>(dx, dy, T.z[q], zj, fx, fy, fz, own[q][0],
                                                       own[q][1], own[q][2], k, acc[q][0],
                                                       acc[q][1], acc[q][2], cs[0], cs[1], cs[2],
                                                       tq, own[q] + 3);
      else
        pair_velocity_sym<double, true, TORQUE, WALL>(dx, dy, T.z[q], zj, fx, fy, fz, own[q][0],
                                                      own[q][1], own[q][2], k, acc[q][0],
                                                      acc[q][1], acc[q][2], cs[0], cs[1], cs[2],
                                                      tq, own[q] + 3);
    });
  }
}

// The targets' own weighted force and torque (zero for rows past the end).
template <int TPT, typename Real>
__device__ __forceinline__ void load_own(const Real *__restrict__ src, int64_t n, int64_t stride,
                                         int64_t first, bool torque, Real (&own)[TPT][6]) {
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int64_t r = first + q * kBlock + threadIdx.x;
    const bool on = r < n;
#pragma unroll
    for (int c = 0; c < 6; ++c)
      own[q][c] = on && (c < 3 || torque) ? src[c * stride + r] : Real(0);
  }
}

// ---- diagonal tile pairs: each unordered pair of the tile once -----------------------------
//
// A diagonal tile pair (I, I) with source part h (a multiple of 64 spheres) covers the pairs of
// the tile's own spheres.  In 64-blocks: target block tb (q * 4 + wavefront) and source block
// sb are taken in both directions when tb < sb, skipped when tb > sb (that block pair is taken
// by the part holding tb's spheres as sources), and on the block diagonal tb = sb over rotation
// steps 0..32 only: step k pairs lane l with source lane l + k, so steps 1..31 meet each pair of
// the block once, step 32 meets the pairs (l, l + 32) twice (lanes below 32 keep them) and step 0
// is the self pair, taken in one direction.  The column sums are rows of the same tile and are
// added into the targets' own sums.

// One rotation step of a diagonal tile (sym_step with a per-target-block mode: 0 skip, 1 both
// directions, 2 the block diagonal).
template <int TPT, bool TORQUE, bool WALL, bool PERIODIC>
__device__ __forceinline__ void sym_step_diag(const LdsF<TORQUE> &L, int j, bool valid, int step,
                                              const int (&mode)[TPT], const TargetsF<TPT> &T,
                                              const float (&own)[TPT][6],
                                              const PairConsts<float> &k, float (&acc)[TPT][3],
                                              float (&cs)[3]) {
  const int lane = threadIdx.x & 63;
  const float xjh = L.xh[j], xjl = L.xl[j], yjh = L.yh[j], yjl = L.yl[j], zj = L.z[j];
  const float f0 = L.f[0][j], f1 = L.f[1][j], f2 = L.f[2][j];
  float t0[3] = {0.f, 0.f, 0.f};
  if (TORQUE) {
#pragma unroll
    for (int c = 0; c < 3; ++c) t0[c] = L.t[c][j];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) cs[c] = wave_rol1(cs[c]);
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    if (mode[q] == 0 || (mode[q] == 2 && step > 32)) continue;
    const bool v = valid && !(mode[q] == 2 && step == 32 && lane >= 32);
    const bool back = v && !(mode[q] == 2 && step == 0);
    const float fx = v ? f0 : 0.f, fy = v ? f1 : 0.f, fz = v ? f2 : 0.f;
    float tq[3], g[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) tq[c] = v ? t0[c] : 0.f;
#pragma unroll
    for (int c = 0; c < 6; ++c) g[c] = back ? own[q][c] : 0.f;
    const float dx0 = (T.xh[q] - xjh) + (T.xl[q] - xjl);
    const float dy0 = (T.yh[q] - yjh) + (T.yl[q] - yjl);
    for_images<PERIODIC>(dx0, dy0, k, [&](float dx, float dy) {
      const float dz = T.z[q] - zj;
      if (dx * dx + dy * dy + dz * dz < float(kFourA2))
        pair_velocity_sym<float, false, TORQUE, WALL>(dx, dy, T.z[q], zj, fx, fy, fz, g[0], g[1],
                                                      g[2], k, acc[q][0], acc[q][1], acc[q][2],
                                                      cs[0], cs[1], cs[2], tq, g + 3);
      else
        pair_velocity_sym<float, true, TORQUE, WALL>(dx, dy, T.z[q], zj, fx, fy, fz, g[0], g[1],
                                                     g[2], k, acc[q][0], acc[q][1], acc[q][2],
                                                     cs[0], cs[1], cs[2], tq, g + 3);
    });
  }
}

template <int TPT, bool TORQUE, bool WALL, bool PERIODIC>
__device__ __forceinline__ void sym_step_diag(const LdsD<TORQUE> &L, int j, bool valid, int step,
                                              const int (&mode)[TPT], const TargetsD<TPT> &T,
                                              const double (&own)[TPT][6],
                                              const PairConsts<double> &k, double (&acc)[TPT][3],
                                              double (&cs)[3]) {
  const int lane = threadIdx.x & 63;
  const double xj = L.x[j], yj = L.y[j], zj = L.z[j];
  const double f0 = L.f[0][j], f1 = L.f[1][j], f2 = L.f[2][j];
  double t0[3] = {0.0, 0.0, 0.0};
  if (TORQUE) {
#pragma unroll
    for (int c = 0; c < 3; ++c) t0[c] = L.t[c][j];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) cs[c] = wave_rol1(cs[c]);
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    if (mode[q] == 0 || (mode[q] == 2 && step > 32)) continue;
    const bool v = valid && !(mode[q] == 2 && step == 32 && lane >= 32);
    const bool back = v && !(mode[q] == 2 && step == 0);
    const double fx = v ? f0 : 0.0, fy = v ? f1 : 0.0, fz = v ? f2 : 0.0;
    double tq[3], g[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) tq[c] = v ? t0[c] : 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) g[c] = back ? own[q][c] : 0.0;
    for_images<PERIODIC>(T.x[q] - xj, T.y[q] - yj, k, [&](double dx, double dy) {
      const double dz = T.z[q] - zj;
      if (dx * dx + dy * dy + dz * dz < kFourA2)
        pair_velocity_sym<double, false, TORQUE, WALL>(dx, dy, T.z[q], zj, fx, fy, fz, g[0],
                                                       g[1], g[2], k, acc[q][0], acc[q][1],
                                                       acc[q][2], cs[0], cs[1], cs[2], tq, g + 3);
      else
        pair_velocity_sym<double, true, TORQUE, WALL>(dx, dy, T.z[q], zj, fx, fy, fz, g[0], g[1],
                                                      g[2], k, acc[q][0], acc[q][1], acc[q][2],
                                                      cs[0], cs[1], cs[2], tq, g + 3);
    });
  }
}

// Mode of each of the lane's target blocks against source block sb (see above); returns the
// number of rotation steps the block needs (64 if some target block takes both directions, 33
// if only the block diagonal, 0 if none).
template <int TPT>
__device__ __forceinline__ int diag_modes(int sb, int (&mode)[TPT]) {
  const int wave = threadIdx.x / 64;
  int steps = 0;
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int tb = q * (kBlock / 64) + wave;
    mode[q] = tb < sb ? 1 : (tb == sb ? 2 : 0);
    steps = max(steps, mode[q] == 1 ? 64 : (mode[q] == 2 ? 33 : 0));
  }
  return steps;
}

// Sources [jb, je) (part h of tile I, starting a multiple of 64 into the tile at jt) against the
// tile's own targets, each unordered pair once; sums into T (row sums and the column sums of
// these sources, which are rows of the same tile).
template <int TPT, bool TORQUE, bool WALL, bool PERIODIC>
__device__ __forceinline__ void sym_diag_tile(const SymArgs &a, const GeomF &g,
                                              const float *__restrict__ src,
                                              const PairConsts<float> &k, int64_t first,
                                              int64_t jb, int64_t je, LdsF<TORQUE> &L,
                                              float (&col)[kWaves][kBlock][3], TargetsF<TPT> &T) {
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  float own[TPT][6];
  load_own<TPT>(src, a.n, a.stride, first, TORQUE, own);
  for (int64_t t0 = jb; t0 < je; t0 += kBlock) {
    const int cnt = int(min<int64_t>(kBlock, je - t0));
    __syncthreads();
    if (tid < cnt) {
      const int64_t j = t0 + tid;
      L.xh[tid] = g.xh[j];
      L.xl[tid] = g.xl[j];
      L.yh[tid] = g.yh[j];
      L.yl[tid] = g.yl[j];
      L.z[tid] = g.z[j];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        L.f[c][tid] = src[c * a.stride + j];
        if (TORQUE) L.t[c][tid] = src[(3 + c) * a.stride + j];
      }
    }
    __syncthreads();
    float acc[TPT][3];
#pragma unroll
    for (int q = 0; q < TPT; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.f;
    const int off = int(t0 - first);   // the LDS tile's first source, within the tile
    for (int blk = 0; blk < cnt; blk += 64) {
      const int nb = min(64, cnt - blk);
      int mode[TPT];
      const int steps = diag_modes<TPT>((off + blk) / 64, mode);
      float cs[3] = {0.f, 0.f, 0.f};
      for (int step = 0; step < steps; ++step) {
        const int sl = (lane + step) & 63;
        sym_step_diag<TPT, TORQUE, WALL, PERIODIC>(L, blk + (sl < nb ? sl : 0), sl < nb, step,
                                                   mode, T, own, k, acc, cs);
      }
      // after step s lane l holds the sums of source (l + s) mod 64
      const int sl = (lane + (steps > 0 ? steps - 1 : 0)) & 63;
      if (sl < nb) {
        col[wave][blk + sl][0] = steps > 0 ? cs[0] : 0.f;
        col[wave][blk + sl][1] = steps > 0 ? cs[1] : 0.f;
        col[wave][blk + sl][2] = steps > 0 ? cs[2] : 0.f;
      }
    }
#pragma unroll
    for (int q = 0; q < TPT; ++q)
#pragma unroll
      for (int d = 0; d < 3; ++d) kahan_add(T.s[q][d], T.c[q][d], acc[q][d]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
      const int idx = q * kBlock + tid - off;
      if (idx >= 0 && idx < cnt)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          double v = 0.0;
#pragma unroll
          for (int w = 0; w < kWaves; ++w) v += double(col[w][idx][d]);
          kahan_add(T.s[q][d], T.c[q][d], float(v));
        }
    }
  }
}

template <int TPT, bool TORQUE, bool WALL, bool PERIODIC>
__device__ __forceinline__ void sym_diag_tile(const SymArgs &a, const GeomD &g,
                                              const double *__restrict__ src,
                                              const PairConsts<double> &k, int64_t first,
                                              int64_t jb, int64_t je, LdsD<TORQUE> &L,
                                              double (&col)[kWaves][kBlock][3], TargetsD<TPT> &T) {
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  double own[TPT][6];
  load_own<TPT>(src, a.n, a.stride, first, TORQUE, own);
  for (int64_t t0 = jb; t0 < je; t0 += kBlock) {
    const int cnt = int(min<int64_t>(kBlock, je - t0));
    __syncthreads();
    if (tid < cnt) {
      const int64_t j = t0 + tid;
      L.x[tid] = g.x[j];
      L.y[tid] = g.y[j];
      L.z[tid] = g.z[j];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        L.f[c][tid] = src[c * a.stride + j];
        if (TORQUE) L.t[c][tid] = src[(3 + c) * a.stride + j];
      }
    }
    __syncthreads();
    const int off = int(t0 - first);
    for (int blk = 0; blk < cnt; blk += 64) {
      const int nb = min(64, cnt - blk);
      int mode[TPT];
      const int steps = diag_modes<TPT>((off + blk) / 64, mode);
      double cs[3] = {0.0, 0.0, 0.0};
      for (int step = 0; step < steps; ++step) {
        const int sl = (lane + step) & 63;
        sym_step_diag<TPT, TORQUE, WALL, PERIODIC>(L, blk + (sl < nb ? sl : 0), sl < nb, step,
                                                   mode, T, own, k, T.u, cs);
      }
      const int sl = (lane + (steps > 0 ? steps - 1 : 0)) & 63;
      if (sl < nb) {
        col[wave][blk + sl][0] = steps > 0 ? cs[0] : 0.0;
        col[wave][blk + sl][1] = steps > 0 ? cs[1] : 0.0;
        col[wave][blk + sl][2] = steps > 0 ? cs[2] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
      const int idx = q * kBlock + tid - off;
      if (idx >= 0 && idx < cnt)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          double v = 0.0;
#pragma unroll
          for (int w = 0; w < kWaves; ++w) v += col[w][idx][d];
          T.u[q][d] += v;
        }
    }
  }
}

// Tile pair (I, J), I <= J, of linear index Lp, source part h, of one system: `g`, `src` and
// `partial` already point at the system's first sphere and first partial; the slots follow
// `pm`.  The mixed kernels store their partial sums as float32 (the compensated row sums and
// the float64 column sums over the wavefronts, rounded once).  Every lane of the workgroup
// must call this.
template <int TPT, bool TORQUE, bool WALL, bool PERIODIC>
__device__ __forceinline__ void sym_tile_pair(const SymArgs &a, const GeomF &g,
                                              const float *__restrict__ src,
                                              const PairConsts<float> &k,
                                              float *__restrict__ partial, const PartMap &pm,
                                              int64_t Lp, int64_t I, int64_t J, int64_t h,
                                              LdsF<TORQUE> &L, float (&col)[kWaves][kBlock][3]) {
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int64_t n = a.n;
  const int64_t first = I * a.ts;
  TargetsF<TPT> T;
  load_targets<TPT>(g, first, n, first, T);
  // source part h of tile J
  const int64_t jt = J * a.ts, part = a.ts / a.nsplit;
  const int64_t jb = jt + h * part, je = min(n, jb + part);
  if (I == J) {
    if (part % 64 == 0)
      sym_diag_tile<TPT, TORQUE, WALL, PERIODIC>(a, g, src, k, first, jb, je, L, col, T);
    else
      sources_mixed<TORQUE, TPT, WALL, PERIODIC>(g, src, a.stride, jb, je, k, L, T);
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
      const int64_t local = q * kBlock + tid;
      if (first + local < n)
#pragma unroll
        for (int d = 0; d < 3; ++d)
          partial[part_elem(pm, Lp, h, 0, d, local)] =
              float(double(T.s[q][d]) - double(T.c[q][d]));
    }
    return;
  }
  float own[TPT][6];
  load_own<TPT>(src, n, a.stride, first, TORQUE, own);
  for (int64_t t0 = jb; t0 < je; t0 += kBlock) {
    const int cnt = int(min<int64_t>(kBlock, je - t0));
    __syncthreads();
    if (tid < cnt) {
      const int64_t j = t0 + tid;
      L.xh[tid] = g.xh[j];
      L.xl[tid] = g.xl[j];
      L.yh[tid] = g.yh[j];
      L.yl[tid] = g.yl[j];
      L.z[tid] = g.z[j];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        L.f[c][tid] = src[c * a.stride + j];
        if (TORQUE) L.t[c][tid] = src[(3 + c) * a.stride + j];
      }
    }
    __syncthreads();
    float acc[TPT][3];
#pragma unroll
    for (int q = 0; q < TPT; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.f;
    for (int blk = 0; blk < cnt; blk += 64) {
      const int nb = min(64, cnt - blk);
      float cs[3] = {0.f, 0.f, 0.f};   // rotating per-source sums
      if (nb == 64) {
#pragma unroll 2
        for (int step = 0; step < 64; ++step)
          sym_step<TPT, TORQUE, WALL, PERIODIC>(L, blk + ((lane + step) & 63), true, T, own, k,
                                                acc, cs);
      } else {
        for (int step = 0; step < 64; ++step) {
          const int sl = (lane + step) & 63;
          sym_step<TPT, TORQUE, WALL, PERIODIC>(L, blk + (sl < nb ? sl : 0), sl < nb, T, own, k,
                                                acc, cs);
        }
      }
      const int sl = (lane + 63) & 63;
      if (sl < nb) {
        col[wave][blk + sl][0] = cs[0];
        col[wave][blk + sl][1] = cs[1];
        col[wave][blk + sl][2] = cs[2];
      }
    }
#pragma unroll
    for (int q = 0; q < TPT; ++q)
#pragma unroll
      for (int d = 0; d < 3; ++d) kahan_add(T.s[q][d], T.c[q][d], acc[q][d]);
    __syncthreads();
    if (tid < cnt) {
      const int64_t l = t0 - jt + tid;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) v += double(col[w][tid][d]);
        partial[part_elem(pm, Lp, pm.nsplit, 0, d, l)] = float(v);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int64_t local = q * kBlock + tid;
    if (first + local < n)
#pragma unroll
      for (int d = 0; d < 3; ++d)
        partial[part_elem(pm, Lp, h, 0, d, local)] = float(double(T.s[q][d]) - double(T.c[q][d]));
  }
}

template <int TPT, bool TORQUE, bool WALL, bool PERIODIC>
__device__ __forceinline__ void sym_tile_pair(const SymArgs &a, const GeomD &g,
                                              const double *__restrict__ src,
                                              const PairConsts<double> &k,
                                              double *__restrict__ partial, const PartMap &pm,
                                              int64_t Lp, int64_t I, int64_t J, int64_t h,
                                              LdsD<TORQUE> &L, double (&col)[kWaves][kBlock][3]) {
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int64_t n = a.n;
  const int64_t first = I * a.ts;
  TargetsD<TPT> T;
  load_targets<TPT>(g, first, n, first, T);
  // source part h of tile J
  const int64_t jt = J * a.ts, part = a.ts / a.nsplit;
  const int64_t jb = jt + h * part, je = min(n, jb + part);
  if (I == J) {
    if (part % 64 == 0)
      sym_diag_tile<TPT, TORQUE, WALL, PERIODIC>(a, g, src, k, first, jb, je, L, col, T);
    else
      sources_f64<TORQUE, TPT, WALL, PERIODIC>(g, src, a.stride, jb, je, k, L, T);
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
      const int64_t local = q * kBlock + tid;
      if (first + local < n)
#pragma unroll
        for (int d = 0; d < 3; ++d) partial[part_elem(pm, Lp, h, 0, d, local)] = T.u[q][d];
    }
    return;
  }
  double own[TPT][6];
  load_own<TPT>(src, n, a.stride, first, TORQUE, own);
  for (int64_t t0 = jb; t0 < je; t0 += kBlock) {
    const int cnt = int(min<int64_t>(kBlock, je - t0));
    __syncthreads();
    if (tid < cnt) {
      const int64_t j = t0 + tid;
      L.x[tid] = g.x[j];
      L.y[tid] = g.y[j];
      L.z[tid] = g.z[j];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        L.f[c][tid] = src[c * a.stride + j];
        if (TORQUE) L.t[c][tid] = src[(3 + c) * a.stride + j];
      }
    }
    __syncthreads();
    for (int blk = 0; blk < cnt; blk += 64) {
      const int nb = min(64, cnt - blk);
      double cs[3] = {0.0, 0.0, 0.0};   // rotating per-source sums
      if (nb == 64) {
#pragma unroll 2
        for (int step = 0; step < 64; ++step)
          sym_step<TPT, TORQUE, WALL, PERIODIC>(L, blk + ((lane + step) & 63), true, T, own, k,
                                                T.u, cs);
      } else {
        for (int step = 0; step < 64; ++step) {
          const int sl = (lane + step) & 63;
          sym_step<TPT, TORQUE, WALL, PERIODIC>(L, blk + (sl < nb ? sl : 0), sl < nb, T, own, k,
                                                T.u, cs);
        }
      }
      const int sl = (lane + 63) & 63;
      if (sl < nb) {
        col[wave][blk + sl][0] = cs[0];
        col[wave][blk + sl][1] = cs[1];
        col[wave][blk + sl][2] = cs[2];
      }
    }
    __syncthreads();
    if (tid < cnt) {
      const int64_t l = t0 - jt + tid;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) v += col[w][tid][d];
        partial[part_elem(pm, Lp, pm.nsplit, 0, d, l)] = v;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int64_t local = q * kBlock + tid;
    if (first + local < n)
#pragma unroll
      for (int d = 0; d < 3; ++d) partial[part_elem(pm, Lp, h, 0, d, local)] = T.u[q][d];
  }
}

// One workgroup per (tile pair, source part) of the chunk [pm.L0, pm.L0 + gridDim.x / nsplit).
template <int TPT, bool TORQUE, bool WALL, bool PERIODIC>
__global__ __launch_bounds__(kBlock) void pair_kernel_mixed_sym(SymArgs a, PartMap pm, GeomF g,
                                                                const float *__restrict__ src,
                                                                PairConsts<float> k_arg,
                                                                float *__restrict__ partial) {
  const PairConsts<float> k = vgpr_consts(k_arg);
  if (a.skip && *a.skip) return;
  __shared__ LdsF<TORQUE> L;
  __shared__ float col[kWaves][kBlock][3];
  int64_t I, J;
  const int64_t Lp = pm.L0 + int64_t(blockIdx.x) / a.nsplit;
  tri_decode(Lp, a.nt, I, J);
  sym_tile_pair<TPT, TORQUE, WALL, PERIODIC>(a, g, src, k, partial, pm, Lp, I, J,
                                             int64_t(blockIdx.x) % a.nsplit, L, col);
}

template <int TPT, bool TORQUE, bool WALL, bool PERIODIC>
__global__ __launch_bounds__(kBlock) void pair_kernel_f64_sym(SymArgs a, PartMap pm, GeomD g,
                                                              const double *__restrict__ src,
                                                              PairConsts<double> k_arg,
                                                              double *__restrict__ partial) {
  const PairConsts<double> k = vgpr_consts(k_arg);
  if (a.skip && *a.skip) return;
  __shared__ LdsD<TORQUE> L;
  __shared__ double col[kWaves][kBlock][3];
  int64_t I, J;
  const int64_t Lp = pm.L0 + int64_t(blockIdx.x) / a.nsplit;
  tri_decode(Lp, a.nt, I, J);
  sym_tile_pair<TPT, TORQUE, WALL, PERIODIC>(a, g, src, k, partial, pm, Lp, I, J,
                                             int64_t(blockIdx.x) % a.nsplit, L, col);
}

// kRedGroups threads per (component, row), 64 rows per workgroup (one wavefront per group):
// the partials of the chunk [pm.L0, L1) dealt over the groups (chunk_row_sum_dealt) and the
// group sums added in a fixed order, written to vel on the first chunk and added to it on the
// others; after the last chunk the sum is scaled by H_i / (8 pi eta a).
constexpr int kRedGroups = 8;

template <typename Part>
__global__ __launch_bounds__(64 * kRedGroups) void reduce_sym_chunk(
    SymArgs a, PartMap pm, int64_t L1, int first, int last, const Part *__restrict__ partial,
    const double *__restrict__ h, double scale, double *__restrict__ vel) {
  __shared__ double sh[kRedGroups * 64];
  if (a.skip && *a.skip) return;
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int64_t e = int64_t(blockIdx.x) * 64 + lane;
  const bool live = e < 3 * a.n;
  const int d = live ? int(e / a.n) : 0;
  const int64_t r = live ? e - int64_t(d) * a.n : 0;
  sh[grp * 64 + lane] =
      live ? chunk_row_sum_dealt(partial, pm, a.nt, L1, r / a.ts, r % a.ts, d, grp, kRedGroups)
           : 0.0;
  __syncthreads();
  if (grp != 0 || !live) return;
  double v = sh[lane];
  for (int q = 1; q < kRedGroups; ++q) v += sh[q * 64 + lane];
  if (!first) v += vel[3 * r + d];
  vel[3 * r + d] = last ? scale * h[r] * v : v;
}

// ---- batched systems: persistent workgroups over a cost-ordered item list -------------------

struct BatchArgs {
  const int64_t *offs;   // nsys + 1 prefix sums (device)
  const int4 *items;     // (system, target tile, source chunk, 0), largest first
  int nitems;
  int *counter;          // work counter (reset to 0 before the launch)
  int64_t n;             // total spheres (stride of every array)
  int64_t chunk;         // sources per item
  const int *done;       // optional per-system flags: items of finished systems are skipped
  const int *all_done;   // optional: nonzero once every system is done (the launch returns)
};

// Pull the next item for the workgroup (-1 when the list is exhausted).  Every workgroup
// keeps pulling until the counter passes nitems, so every wave reaches the exit.
__device__ __forceinline__ int next_item(const BatchArgs &b, int *slot) {
  __syncthreads();
  if (threadIdx.x == 0) slot[0] = atomicAdd(b.counter, 1);
  __syncthreads();
  const int it = slot[0];
  return it < b.nitems ? it : -1;
}

template <bool TORQUE, int TPT, bool WALL>
__global__ __launch_bounds__(kBlock) void pair_kernel_f64_batched(BatchArgs b, GeomD g,
                                                                  const double *__restrict__ src,
                                                                  PairConsts<double> k_arg,
                                                                  double *__restrict__ partial) {
  const PairConsts<double> k = vgpr_consts(k_arg);
  __shared__ LdsD<TORQUE> L;
  __shared__ int slot[1];
  if (b.all_done && *b.all_done) return;
  for (int it = next_item(b, slot); it >= 0; it = next_item(b, slot)) {
    const int4 w = b.items[it];
    if (b.done && b.done[w.x]) continue;
    const int64_t s0 = b.offs[w.x], s1 = b.offs[w.x + 1];
    TargetsD<TPT> T;
    const int64_t first = s0 + int64_t(w.y) * (kBlock * TPT);
    load_targets<TPT>(g, first, s1, s0, T);
    const int64_t jb = s0 + int64_t(w.z) * b.chunk;
    sources_f64<TORQUE, TPT, WALL, false>(g, src, b.n, jb, min(s1, jb + b.chunk), k, L, T);
    store_partial<TPT>(T, first, s1, w.z, b.n, 0, partial);
  }
}

template <bool TORQUE, int TPT, bool WALL>
__global__ __launch_bounds__(kBlock) void pair_kernel_mixed_batched(BatchArgs b, GeomF g,
                                                                    const float *__restrict__ src,
                                                                    PairConsts<float> k_arg,
                                                                    double *__restrict__ partial) {
  const PairConsts<float> k = vgpr_consts(k_arg);
  __shared__ LdsF<TORQUE> L;
  __shared__ int slot[1];
  if (b.all_done && *b.all_done) return;
  for (int it = next_item(b, slot); it >= 0; it = next_item(b, slot)) {
    const int4 w = b.items[it];
    if (b.done && b.done[w.x]) continue;
    const int64_t s0 = b.offs[w.x], s1 = b.offs[w.x + 1];
    TargetsF<TPT> T;
    const int64_t first = s0 + int64_t(w.y) * (kBlock * TPT);
    load_targets<TPT>(g, first, s1, s0, T);
    const int64_t jb = s0 + int64_t(w.z) * b.chunk;
    sources_mixed<TORQUE, TPT, WALL, false>(g, src, b.n, jb, min(s1, jb + b.chunk), k, L, T);
    store_partial<TPT>(T, first, s1, w.z, b.n, 0, partial);
  }
}

__global__ void reduce_partials_batched(int64_t n, const int *__restrict__ sys_of,
                                        const int64_t *__restrict__ offs, int64_t chunk,
                                        const int *__restrict__ done,
                                        const double *__restrict__ partial,
                                        const double *__restrict__ h, double scale,
                                        double *__restrict__ vel) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int s = sys_of[r];
  if (done && done[s]) return;
  const int64_t nch = (offs[s + 1] - offs[s] + chunk - 1) / chunk;
  const double w = scale * h[r];
  for (int c = 0; c < 3; ++c) {
    double acc = 0.0;
    for (int64_t q = 0; q < nch; ++q) acc += partial[(q * 3 + c) * n + r];
    vel[3 * r + c] = w * acc;
  }
}

// Symmetric batched product: items are (system, I, J) tile pairs with I <= J; system s owns the
// partial slots from part_base[s] on, laid out as in the single-system symmetric kernel.
struct SymBatchArgs {
  const int64_t *offs;       // nsys + 1 prefix sums (device)
  const int4 *items;         // (system, I, J, 0), largest first
  int nitems;
  int *counter;              // work counter (reset to 0 before the launch)
  int64_t n;                 // total spheres (stride of the source arrays)
  int64_t ts;                // tile size
  const int64_t *part_base;  // first partial slot of each system
  const int *done;           // optional per-system flags: items of finished systems are skipped
  const int *all_done;       // optional: nonzero once every system is done (the launch returns)
  int64_t nsplit;            // source parts per tile pair (items (system, I, J, part))
};

__device__ __forceinline__ SymArgs sym_args_of(const SymBatchArgs &b, int s) {
  const int64_t ns = b.offs[s + 1] - b.offs[s];
  return SymArgs{ns, b.ts, (ns + b.ts - 1) / b.ts, b.n, b.nsplit};
}

__device__ __forceinline__ int next_sym_item(const SymBatchArgs &b, int *slot) {
  __syncthreads();
  if (threadIdx.x == 0) slot[0] = atomicAdd(b.counter, 1);
  __syncthreads();
  const int it = slot[0];
  return it < b.nitems ? it : -1;
}

template <int TPT, bool TORQUE, bool WALL>
__global__ __launch_bounds__(kBlock) void pair_kernel_mixed_sym_batched(
    SymBatchArgs b, GeomF g, const float *__restrict__ src, PairConsts<float> k_arg,
    float *__restrict__ partial) {
  const PairConsts<float> k = vgpr_consts(k_arg);
  __shared__ LdsF<TORQUE> L;
  __shared__ float col[kWaves][kBlock][3];
  __shared__ int slot[1];
  if (b.all_done && *b.all_done) return;
  const PartMap pm{0, b.nsplit, b.ts, 1};
  for (int it = next_sym_item(b, slot); it >= 0; it = next_sym_item(b, slot)) {
    const int4 w = b.items[it];
    if (b.done && b.done[w.x]) continue;
    const int64_t s0 = b.offs[w.x];
    const SymArgs a = sym_args_of(b, w.x);
    sym_tile_pair<TPT, TORQUE, WALL, false>(a, offset_geom(g, s0), src + s0, k,
                                            partial + b.part_base[w.x], pm,
                                            tri_start(w.y, a.nt) + w.z - w.y, w.y, w.z, w.w, L,
                                            col);
  }
}

template <int TPT, bool TORQUE, bool WALL>
__global__ __launch_bounds__(kBlock) void pair_kernel_f64_sym_batched(
    SymBatchArgs b, GeomD g, const double *__restrict__ src, PairConsts<double> k_arg,
    double *__restrict__ partial) {
  const PairConsts<double> k = vgpr_consts(k_arg);
  __shared__ LdsD<TORQUE> L;
  __shared__ double col[kWaves][kBlock][3];
  __shared__ int slot[1];
  if (b.all_done && *b.all_done) return;
  const PartMap pm{0, b.nsplit, b.ts, 1};
  for (int it = next_sym_item(b, slot); it >= 0; it = next_sym_item(b, slot)) {
    const int4 w = b.items[it];
    if (b.done && b.done[w.x]) continue;
    const int64_t s0 = b.offs[w.x];
    const SymArgs a = sym_args_of(b, w.x);
    sym_tile_pair<TPT, TORQUE, WALL, false>(a, offset_geom(g, s0), src + s0, k,
                                            partial + b.part_base[w.x], pm,
                                            tri_start(w.y, a.nt) + w.z - w.y, w.y, w.z, w.w, L,
                                            col);
  }
}

// System s's partials start at part_base[s] and cover its whole triangle (one chunk).
template <typename Part>
__global__ void reduce_partials_sym_batched(SymBatchArgs b, const int *__restrict__ sys_of,
                                            const Part *__restrict__ partial,
                                            const double *__restrict__ h, double scale,
                                            double *__restrict__ vel) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;   // (component, row)
  if (e >= 3 * b.n) return;
  const int d = int(e / b.n);
  const int64_t r = e - int64_t(d) * b.n;
  const int s = sys_of[r];
  if (b.done && b.done[s]) return;
  const SymArgs a = sym_args_of(b, s);
  const int64_t local = r - b.offs[s];
  const PartMap pm{0, b.nsplit, b.ts, 1};
  vel[3 * r + d] = scale * h[r] *
                   chunk_row_sum(partial + b.part_base[s], pm, a.nt, a.nt * (a.nt + 1) / 2,
                                 local / a.ts, local % a.ts, 0, d);
}

__global__ void fill_sys_of(int nsys, const int64_t *__restrict__ offs, int *__restrict__ sys_of) {
  const int s = blockIdx.x;
  if (s >= nsys) return;
  for (int64_t i = offs[s] + threadIdx.x; i < offs[s + 1]; i += blockDim.x) sys_of[i] = s;
}

__global__ void zero_int(int *p) { p[0] = 0; }

__global__ void finite_flag(int64_t m, const double *__restrict__ v, int *__restrict__ flag) {
  int bad = 0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < m;
       i += int64_t(gridDim.x) * blockDim.x)
    bad |= !isfinite(v[i]);
  if (bad) flag[0] = 1;   // benign race: every writer stores the same value
}


// L with L^2 = diag(M_ii): the self pair (r = 0, R = (0, 0, 2 z~)) applied to e_x and e_z, in
// float64 whatever the product precision; H = 0 keeps L = 1.
template <bool WALL, typename Geom>
__global__ void self_scale(int64_t n, Geom g, PairConsts<double> k, double inv8pieta,
                           double *__restrict__ scale) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double z = double(g.z[i]), w = g.h[i] * g.h[i] * inv8pieta;
  double px = 0.0, py = 0.0, pz = 0.0, nx = 0.0, ny = 0.0, nz = 0.0;
  pair_velocity<double, false, false, WALL>(0.0, 0.0, z, z, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, k, px,
                                            py, pz);
  pair_velocity<double, false, false, WALL>(0.0, 0.0, z, z, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, k, nx,
                                            ny, nz);
  const double dpar = w * px, dperp = w * nz;
  scale[3 * i] = scale[3 * i + 1] = dpar > 0.0 ? sqrt(dpar) : 1.0;
  scale[3 * i + 2] = dperp > 0.0 ? sqrt(dperp) : 1.0;
}

// Calls fn(torque, tpt, wall, periodic) with the four as std::integral_constant values, so
// each launch site names its kernel template once.
template <typename Fn>
void with_variant(bool torque, int tpt, bool wall, bool periodic, Fn &&fn) {
  using T1 = std::true_type;
  using T0 = std::false_type;
  using P2 = std::integral_constant<int, 2>;
  using P1 = std::integral_constant<int, 1>;
  auto by_box = [&](auto t, auto q, auto w) {
    if (periodic)
      fn(t, q, w, T1{});
    else
      fn(t, q, w, T0{});
  };
  auto by_wall = [&](auto t, auto q) {
    if (wall)
      by_box(t, q, T1{});
    else
      by_box(t, q, T0{});
  };
  if (torque) {
    if (tpt == 2)
      by_wall(T1{}, P2{});
    else
      by_wall(T1{}, P1{});
  } else {
    if (tpt == 2)
      by_wall(T0{}, P2{});
    else
      by_wall(T0{}, P1{});
  }
}

inline bool periodic(const rpb_params *p) { return p->lx > 0.0; }

// H-weighted sources of packed geometry `g` into `buf` (6 n values of the pair precision).
int pack_sources_into(rpb_ctx *ctx, const Packed &g, const double *force, const double *torque,
                      void *buf, hipStream_t stream, const int *skip = nullptr) {
  const int64_t n = g.n;
  const bool f64 = g.precision == RPB_FP64;
  const double *h = f64 ? geom_d(g).h : geom_f(g).h;
  if (f64)
    pack_vectors<double><<<blocks_for(n, 256), 256, 0, stream>>>(
        n, h, force, torque, 1.0 / g.a, static_cast<double *>(buf), skip);
  else
    pack_vectors<float><<<blocks_for(n, 256), 256, 0, stream>>>(
        n, h, force, torque, 1.0 / g.a, static_cast<float *>(buf), skip);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

int pack_sources(rpb_ctx *ctx, const Packed &g, const double *force, const double *torque,
                 void **src, hipStream_t stream, const int *skip = nullptr) {
  int st;
  *src = source_buffer(ctx, g, &st);
  if (!*src) return st;
  return pack_sources_into(ctx, g, force, torque, *src, stream, skip);
}

// Source chunking of the ordered kernel: enough workgroups to fill the chip several times
// over (target_wgs), at most max_chunks chunks, each a multiple of kBlock sources.  The
// chunks depend on n only (not on the row range), so every target sums its sources in the
// same order whichever rows are requested: row shards concatenate to the full product bitwise.
inline int64_t ordered_chunk(int64_t n, int tpt, int target_wgs, int64_t max_chunks) {
  const int64_t per_wg = int64_t(kBlock) * tpt;
  const int64_t tiles_full = (n + per_wg - 1) / per_wg;
  int64_t nchunks = std::max<int64_t>(1, (int64_t(target_wgs) + tiles_full - 1) / tiles_full);
  nchunks = std::min(nchunks, std::max<int64_t>(1, max_chunks));
  int64_t chunk = (n + nchunks - 1) / nchunks;
  return std::max<int64_t>(kBlock, (chunk + kBlock - 1) / kBlock * kBlock);
}

// Ordered pair kernel over rows [row0, row0 + nrows) into `part` (nchunks x 3 x nrows
// doubles), then the fixed-order reduction into vel.  `record` brackets the pair kernel with
// the context's timing events.
int ordered_product(rpb_ctx *ctx, const rpb_params *p, const Packed &g, const void *src,
                    bool has_t, int tpt, int64_t chunk, int64_t row0, int64_t nrows,
                    double *part, double *vel, hipStream_t stream, const int *skip, bool record) {
  const int64_t n = g.n;
  const bool f64 = g.precision == RPB_FP64;
  const int64_t per_wg = int64_t(kBlock) * tpt;
  const int64_t tiles = (nrows + per_wg - 1) / per_wg;
  const int64_t nchunks = (n + chunk - 1) / chunk;
  if (tiles > 0x7fffffff || nchunks > 65535)
    return fail(ctx, RPB_EINVAL, "problem too large for one launch (n = %lld)", (long long)n);
  PairArgs args{n, row0, nrows, chunk, skip};
  const dim3 grid{unsigned(tiles), unsigned(nchunks), 1u};
  hipEvent_t t0 = nullptr;
  if (record) RPB_TRY(timing_begin(ctx, stream, &t0));
  with_variant(has_t, tpt, p->wall != 0, periodic(p), [&](auto T, auto P, auto W, auto B) {
    constexpr bool kT = decltype(T)::value, kW = decltype(W)::value, kB = decltype(B)::value;
    constexpr int kP = decltype(P)::value;
    if (f64)
      pair_kernel_f64<kT, kP, kW, kB><<<grid, kBlock, 0, stream>>>(
          args, geom_d(g), static_cast<const double *>(src),
          make_pair_consts<double>(p->lx / p->a, p->ly / p->a), part);
    else
      pair_kernel_mixed<kT, kP, kW, kB><<<grid, kBlock, 0, stream>>>(
          args, geom_f(g), static_cast<const float *>(src),
          make_pair_consts<float>(p->lx / p->a, p->ly / p->a), part);
  });
  RPB_LAUNCHED(ctx);
  if (record)
    RPB_TRY(timing_end(ctx, stream, t0, double(nrows) * double(n),
                       (f64 ? 0 : 2) + (has_t ? 1 : 0)));
  const double *h = f64 ? geom_d(g).h : geom_f(g).h;
  const double scale = 1.0 / (8.0 * M_PI * p->eta * p->a);
  reduce_partials<<<blocks_for(nrows, 256), 256, 0, stream>>>(nrows, int(nchunks), part,
                                                              h + row0, scale, vel, skip);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

}  // namespace

int check_finite(rpb_ctx *ctx, const double *pos, int64_t n, hipStream_t stream) {
  int st;
  char *small = static_cast<char *>(workspace(ctx, WS_SMALL, kSmallBytes, &st));
  if (!small) return st;
  int *f = reinterpret_cast<int *>(small + kSmallFiniteFlag);
  zero_int<<<1, 1, 0, stream>>>(f);
  RPB_LAUNCHED(ctx);
  const int64_t m = 3 * n;
  const unsigned nb = unsigned(std::min<int64_t>(1024, (m + 255) / 256));
  finite_flag<<<nb, 256, 0, stream>>>(m, pos, f);
  RPB_LAUNCHED(ctx);
  int *host = static_cast<int *>(host_scratch(ctx));
  RPB_HIP(ctx, hipMemcpyAsync(host, f, sizeof(int), hipMemcpyDeviceToHost, stream));
  RPB_HIP(ctx, hipStreamSynchronize(stream));
  if (host[0]) return fail(ctx, RPB_ENONFINITE, "positions contain NaN or Inf");
  return RPB_OK;
}

int check_output(rpb_ctx *ctx, const double *v, int64_t m, hipStream_t stream, const char *what) {
  if (!ctx->check_output || m <= 0) return RPB_OK;
  int st;
  char *small = static_cast<char *>(workspace(ctx, WS_SMALL, kSmallBytes, &st));
  if (!small) return st;
  int *f = reinterpret_cast<int *>(small + kSmallFiniteFlag);
  zero_int<<<1, 1, 0, stream>>>(f);
  RPB_LAUNCHED(ctx);
  const unsigned nb = unsigned(std::min<int64_t>(1024, (m + 255) / 256));
  finite_flag<<<nb, 256, 0, stream>>>(m, v, f);
  RPB_LAUNCHED(ctx);
  int *host = static_cast<int *>(host_scratch(ctx));
  RPB_HIP(ctx, hipMemcpyAsync(host, f, sizeof(int), hipMemcpyDeviceToHost, stream));
  RPB_HIP(ctx, hipStreamSynchronize(stream));
  if (host[0]) return fail(ctx, RPB_ENONFINITE, "%s contains NaN or Inf", what);
  return RPB_OK;
}

int check_finite_begin(rpb_ctx *ctx, const double *pos, int64_t n, hipStream_t stream) {
  if (ctx->fin_live) {   // a copy left in flight by a call that failed before its _end
    RPB_HIP(ctx, hipEventSynchronize(ctx->fin_ev));
    ctx->fin_live = false;
  }
  int st;
  char *small = static_cast<char *>(workspace(ctx, WS_SMALL, kSmallBytes, &st));
  if (!small) return st;
  int *f = reinterpret_cast<int *>(small + kSmallFiniteFlag);
  zero_int<<<1, 1, 0, stream>>>(f);
  RPB_LAUNCHED(ctx);
  const int64_t m = 3 * n;
  const unsigned nb = unsigned(std::min<int64_t>(1024, (m + 255) / 256));
  finite_flag<<<nb, 256, 0, stream>>>(m, pos, f);
  RPB_LAUNCHED(ctx);
  if (!ctx->fin_ev) RPB_HIP(ctx, hipEventCreateWithFlags(&ctx->fin_ev, hipEventDisableTiming));
  int *host = reinterpret_cast<int *>(static_cast<char *>(host_scratch(ctx)) + kHostFiniteOffset);
  RPB_HIP(ctx, hipMemcpyAsync(host, f, sizeof(int), hipMemcpyDeviceToHost, stream));
  RPB_HIP(ctx, hipEventRecord(ctx->fin_ev, stream));
  ctx->fin_live = true;
  return RPB_OK;
}

int check_finite_end(rpb_ctx *ctx) {
  if (!ctx->fin_live) return fail(ctx, RPB_EDEVICE, "position check was not started");
  RPB_HIP(ctx, hipEventSynchronize(ctx->fin_ev));
  ctx->fin_live = false;
  const int *host =
      reinterpret_cast<const int *>(static_cast<char *>(host_scratch(ctx)) + kHostFiniteOffset);
  if (host[0]) return fail(ctx, RPB_ENONFINITE, "positions contain NaN or Inf");
  return RPB_OK;
}

size_t packed_geometry_bytes(int64_t n, int precision) { return geom_bytes(n, precision); }

int pack_geometry(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos, Slot slot,
                  Packed *out, hipStream_t stream) {
  int st;
  void *buf = workspace(ctx, slot, geom_bytes(n, p->precision), &st);
  if (!buf) return st;
  return pack_geometry_into(ctx, p, n, pos, buf, out, stream);
}

int pack_geometry_into(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                       void *buf, Packed *out, hipStream_t stream) {
  out->n = n;
  out->a = p->a;
  out->precision = p->precision;
  out->geom = buf;
  if (p->precision == RPB_FP64) {
    pack_geometry_f64<<<blocks_for(n, 256), 256, 0, stream>>>(n, pos, p->a, p->wall,
                                                              static_cast<double *>(buf));
  } else {
    double *h = static_cast<double *>(buf);
    pack_geometry_mixed<<<blocks_for(n, 256), 256, 0, stream>>>(
        n, pos, p->a, p->wall, h, reinterpret_cast<float *>(h + n));
  }
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

int block_diag_scale(rpb_ctx *ctx, const rpb_params *p, const Packed &g, double *scale,
                     hipStream_t stream) {
  const int64_t n = g.n;
  if (n == 0) return RPB_OK;
  const auto k = make_pair_consts<double>();
  const double inv = 1.0 / (8.0 * M_PI * p->eta * p->a);
  const unsigned nb = blocks_for(n, 256);
  if (g.precision == RPB_FP64) {
    if (p->wall)
      self_scale<true><<<nb, 256, 0, stream>>>(n, geom_d(g), k, inv, scale);
    else
      self_scale<false><<<nb, 256, 0, stream>>>(n, geom_d(g), k, inv, scale);
  } else {
    if (p->wall)
      self_scale<true><<<nb, 256, 0, stream>>>(n, geom_f(g), k, inv, scale);
    else
      self_scale<false><<<nb, 256, 0, stream>>>(n, geom_f(g), k, inv, scale);
  }
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

// Small systems have few tile pairs: their sources are split into parts (each of at least
// 128 spheres, one workgroup per part) until the grid has about kSplitWorkgroups workgroups;
// systems of one or a few tiles go on splitting, down to parts of 8 sources, until there are
// at least kMinWorkgroups (a 256-sphere system is one tile pair: 2 to 4 workgroups otherwise).
constexpr int64_t kSplitWorkgroups = 4096;
constexpr int64_t kMinWorkgroups = 64;
inline int64_t sym_nsplit(int64_t n, int64_t ts) {
  const int64_t nt = (n + ts - 1) / ts;
  const int64_t pairs = nt * (nt + 1) / 2;
  int64_t q = 1;
  while (pairs * q < kSplitWorkgroups && ts / (2 * q) >= 128) q *= 2;
  while (pairs * q < kMinWorkgroups && ts / (2 * q) >= 8) q *= 2;
  return q;
}

// Partials of one persistent batched launch of the symmetric kernel (every system's triangle at
// once); larger batches take the ordered items.
constexpr size_t kMaxBatchSymBytes = size_t(4) << 30;

// Calls fn(torque, tpt, wall, periodic) for the symmetric kernel, which also takes 4 targets
// per lane (tiles of 1,024 spheres).
template <typename Fn>
void with_sym_variant(bool torque, int tpt, bool wall, bool periodic, Fn &&fn) {
  if (tpt == 4) {
    using P4 = std::integral_constant<int, 4>;
    auto by_box = [&](auto t, auto w) {
      if (periodic)
        fn(t, P4{}, w, std::true_type{});
      else
        fn(t, P4{}, w, std::false_type{});
    };
    auto by_wall = [&](auto t) {
      if (wall)
        by_box(t, std::true_type{});
      else
        by_box(t, std::false_type{});
    };
    if (torque)
      by_wall(std::true_type{});
    else
      by_wall(std::false_type{});
    return;
  }
  with_variant(torque, tpt, wall, periodic, fn);
}

// Whole-system product with one evaluation per unordered pair.  The triangle of tile pairs is
// walked in chunks whose partials fit the context's limit (512 MiB: one chunk up to about
// 150,000 spheres in mixed precision and 100,000 in float64 at 2 targets per lane), each
// chunk's pair kernel followed by its reduction into vel, so the workspace stays bounded
// whatever n.  The timing record spans the pair kernels of all chunks.
int matvec_symmetric(rpb_ctx *ctx, const rpb_params *p, const Packed &g, const void *src,
                     bool torque, const double *h, int tpt, double *vel, hipStream_t stream,
                     const int *skip) {
  const int64_t n = g.n;
  const bool f64 = g.precision == RPB_FP64;
  SymArgs a{n, int64_t(kBlock) * tpt, 0, n};
  a.skip = skip;
  a.nt = (n + a.ts - 1) / a.ts;
  a.nsplit = sym_nsplit(n, a.ts);
  const int64_t pairs = a.nt * (a.nt + 1) / 2;
  const size_t esz = f64 ? sizeof(double) : sizeof(float);
  const int64_t per = chunk_pairs(pairs, a.nsplit, 1, a.ts, esz, ctx->chunk_bytes);
  int st;
  void *part = workspace(ctx, WS_PART, size_t(part_elems(per, a.nsplit, 1, a.ts)) * esz, &st);
  if (!part) return st;
  const double scale = 1.0 / (8.0 * M_PI * p->eta * p->a);
  hipEvent_t t0;
  RPB_TRY(timing_begin(ctx, stream, &t0));
  for (int64_t L0 = 0; L0 < pairs; L0 += per) {
    const int64_t L1 = std::min(pairs, L0 + per);
    const PartMap pm{L0, a.nsplit, a.ts, 1};
    const unsigned grid = unsigned((L1 - L0) * a.nsplit);
    with_sym_variant(torque, tpt, p->wall != 0, periodic(p), [&](auto T, auto P, auto W, auto B) {
      constexpr bool kT = decltype(T)::value, kW = decltype(W)::value, kB = decltype(B)::value;
      constexpr int kP = decltype(P)::value;
      if (f64)
        pair_kernel_f64_sym<kP, kT, kW, kB><<<grid, kBlock, 0, stream>>>(
            a, pm, geom_d(g), static_cast<const double *>(src),
            make_pair_consts<double>(p->lx / p->a, p->ly / p->a), static_cast<double *>(part));
      else
        pair_kernel_mixed_sym<kP, kT, kW, kB><<<grid, kBlock, 0, stream>>>(
            a, pm, geom_f(g), static_cast<const float *>(src),
            make_pair_consts<float>(p->lx / p->a, p->ly / p->a), static_cast<float *>(part));
    });
    RPB_LAUNCHED(ctx);
    if (L1 == pairs)
      RPB_TRY(timing_end(ctx, stream, t0, double(n) * double(n),
                         (f64 ? 0 : 2) + (torque ? 1 : 0)));
    const int first = L0 == 0, last = L1 == pairs;
    if (f64)
      reduce_sym_chunk<double><<<blocks_for(3 * n, 64), 64 * kRedGroups, 0, stream>>>(
          a, pm, L1, first, last, static_cast<const double *>(part), h, scale, vel);
    else
      reduce_sym_chunk<float><<<blocks_for(3 * n, 64), 64 * kRedGroups, 0, stream>>>(
          a, pm, L1, first, last, static_cast<const float *>(part), h, scale, vel);
    RPB_LAUNCHED(ctx);
  }
  return RPB_OK;
}

const double *packed_weights(const Packed &g) {
  return g.precision == RPB_FP64 ? geom_d(g).h : geom_f(g).h;
}

void *source_buffer(rpb_ctx *ctx, const Packed &g, int *status) {
  const size_t esz = g.precision == RPB_FP64 ? sizeof(double) : sizeof(float);
  return workspace(ctx, WS_SRC, size_t(6 * g.n) * esz, status);
}

int matvec_prepacked(rpb_ctx *ctx, const rpb_params *p, const Packed &g, const void *src,
                     double *vel, hipStream_t stream, const int *skip) {
  const int64_t n = g.n;
  if (n <= 0) return RPB_OK;
  const bool f64 = g.precision == RPB_FP64;
  const Shape &shape = ctx->tune.s[f64 ? RPB_FP64 : RPB_MIXED];
  if (shape.symmetric)
    return matvec_symmetric(ctx, p, g, src, false, packed_weights(g), shape.tpt, vel, stream,
                            skip);
  const int tpt = std::min(shape.tpt, 2);
  const int64_t chunk = ordered_chunk(n, tpt, shape.target_wgs, 65535);
  const int64_t nchunks = (n + chunk - 1) / chunk;
  int st;
  double *part = static_cast<double *>(
      workspace(ctx, WS_PART, size_t(nchunks) * 3 * size_t(n) * sizeof(double), &st));
  if (!part) return st;
  return ordered_product(ctx, p, g, src, false, tpt, chunk, 0, n, part, vel, stream, skip,
                         true);
}

int matvec_packed(rpb_ctx *ctx, const rpb_params *p, const Packed &g, const double *force,
                  const double *torque, int64_t row0, int64_t nrows, double *vel,
                  hipStream_t stream, const int *skip) {
  const int64_t n = g.n;
  if (nrows <= 0) return RPB_OK;
  const bool has_t = torque != nullptr;
  const bool f64 = g.precision == RPB_FP64;
  void *src;
  RPB_TRY(pack_sources(ctx, g, force, torque, &src, stream, skip));
  const double *h = f64 ? geom_d(g).h : geom_f(g).h;

  const Shape &shape = ctx->tune.s[f64 ? RPB_FP64 : RPB_MIXED];
  if (row0 == 0 && nrows == n && shape.symmetric)
    return matvec_symmetric(ctx, p, g, src, has_t, h, shape.tpt, vel, stream, skip);
  const int tpt = std::min(shape.tpt, 2);   // the ordered kernel takes 1 or 2 targets per lane
  const int64_t chunk = ordered_chunk(n, tpt, shape.target_wgs, 65535);
  const int64_t nchunks = (n + chunk - 1) / chunk;
  int st;
  double *part = static_cast<double *>(
      workspace(ctx, WS_PART, size_t(nchunks) * 3 * size_t(nrows) * sizeof(double), &st));
  if (!part) return st;
  return ordered_product(ctx, p, g, src, has_t, tpt, chunk, row0, nrows, part, vel, stream, skip,
                         true);
}

size_t noalloc_matvec_bytes(int64_t n, int precision, int64_t nchunks) {
  const size_t esz = precision == RPB_FP64 ? sizeof(double) : sizeof(float);
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  return up(geom_bytes(n, precision)) + up(size_t(6 * n) * esz) +
         size_t(nchunks) * 3 * size_t(n) * sizeof(double);
}

int matvec_into(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                const double *force, const double *torque, double *vel, void *buf, size_t bytes,
                hipStream_t stream) {
  const int prec = p->precision;
  const Shape &shape = ctx->tune.s[prec == RPB_FP64 ? RPB_FP64 : RPB_MIXED];
  const size_t fixed = noalloc_matvec_bytes(n, prec, 0);
  const size_t per_chunk = 3 * size_t(n) * sizeof(double);
  if (fixed + per_chunk > bytes)
    return fail(ctx, RPB_EINVAL,
                "n = %lld needs %zu bytes of scratch with one source chunk; the scratch holds %zu",
                (long long)n, fixed + per_chunk, bytes);
  const int tpt = std::min(shape.tpt, 2);   // the ordered kernel takes 1 or 2 targets per lane
  const int64_t chunk =
      ordered_chunk(n, tpt, shape.target_wgs, int64_t((bytes - fixed) / per_chunk));
  char *base = static_cast<char *>(buf);
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  void *geom = base;
  void *src = base + up(geom_bytes(n, prec));
  double *part = reinterpret_cast<double *>(static_cast<char *>(src) +
                                            up(size_t(6 * n) * (prec == RPB_FP64 ? 8 : 4)));
  Packed g;
  RPB_TRY(pack_geometry_into(ctx, p, n, pos, geom, &g, stream));
  RPB_TRY(pack_sources_into(ctx, g, force, torque, src, stream));
  return ordered_product(ctx, p, g, src, torque != nullptr, tpt, chunk, 0, n, part, vel, stream,
                         nullptr, false);
}

// ---- batched -----------------------------------------------------------------------------

int prepare_batch(rpb_ctx *ctx, int32_t nsys, const int64_t *offs, int precision, Batch *b,
                  hipStream_t stream, bool work_items) {
  const Shape &shape = ctx->tune.s[precision == RPB_FP64 ? RPB_FP64 : RPB_MIXED];
  const int tpt = shape.batch_tpt;
  const int64_t chunk = shape.batch_chunk;
  b->nsys = nsys;
  b->n = offs[nsys];
  b->chunk = chunk;
  b->tpt = tpt;
  b->wgs = shape.batch_wgs;
  b->symmetric = shape.batch_symmetric != 0;
  const int64_t per = int64_t(kBlock) * tpt;
  // symmetric items are split into source parts (of at least 128 spheres) until there are
  // about four items per persistent workgroup, for balance at the end of the launch; the
  // partial buffer must stay within the limit of the symmetric kernel
  b->nsplit = 1;
  if (b->symmetric) {
    int64_t pairs = 0;
    for (int s = 0; s < nsys; ++s) {
      const int64_t nt = (offs[s + 1] - offs[s] + per - 1) / per;
      pairs += nt * (nt + 1) / 2;
    }
    while (pairs * b->nsplit < 4 * int64_t(b->wgs) && per / (2 * b->nsplit) >= 128) b->nsplit *= 2;
    while (pairs * b->nsplit < kMinWorkgroups && per / (2 * b->nsplit) >= 8) b->nsplit *= 2;
    const size_t esz = precision == RPB_FP64 ? sizeof(double) : sizeof(float);
    size_t bytes = 0;
    for (int s = 0; s < nsys; ++s) {
      const int64_t nt = (offs[s + 1] - offs[s] + per - 1) / per;
      bytes += size_t(part_elems(nt * (nt + 1) / 2, b->nsplit, 1, per)) * esz;
    }
    // one persistent launch holds every system's partials: beyond the limit the batch takes
    // the ordered items, whose partials grow as O(n)
    if (bytes > kMaxBatchSymBytes) {
      b->symmetric = false;
      b->nsplit = 1;
    }
  }
  b->host_offs.assign(offs, offs + nsys + 1);
  // work items, largest (targets x sources) first; ties keep their generation order.
  // Ordered: (system, target tile, source chunk); symmetric: (system, I, J, part), I <= J.
  std::vector<int4> items;
  std::vector<double> cost;
  std::vector<int64_t> part_base(size_t(nsys), 0);
  int64_t part_elems = 0;
  const int64_t part_len = per / b->nsplit;
  for (int s = 0; s < nsys && work_items; ++s) {
    const int64_t ns = offs[s + 1] - offs[s];
    if (b->symmetric) {
      const int64_t nt = (ns + per - 1) / per;
      part_base[s] = part_elems;
      part_elems += rpb::part_elems(nt * (nt + 1) / 2, b->nsplit, 1, per);
      for (int64_t I = 0; I < nt; ++I)
        for (int64_t J = I; J < nt; ++J)
          for (int64_t q = 0; q < b->nsplit; ++q) {
            const int64_t j0 = J * per + q * part_len;
            items.push_back(int4{s, int(I), int(J), int(q)});
            cost.push_back(double(std::min(per, ns - I * per)) *
                           double(std::max<int64_t>(0, std::min(part_len, ns - j0))));
          }
    } else {
      for (int64_t t = 0; t * per < ns; ++t)
        for (int64_t c = 0; c * chunk < ns; ++c) {
          items.push_back(int4{s, int(t), int(c), 0});
          cost.push_back(double(std::min(per, ns - t * per)) *
                         double(std::min(chunk, ns - c * chunk)));
        }
    }
  }
  b->part_elems = part_elems;
  std::vector<size_t> order(items.size());
  std::iota(order.begin(), order.end(), size_t(0));
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t a, size_t c) { return cost[a] > cost[c]; });
  int64_t max_chunks = 1;
  for (int s = 0; s < nsys; ++s)
    max_chunks = std::max<int64_t>(max_chunks, (offs[s + 1] - offs[s] + chunk - 1) / chunk);
  b->nitems = int(items.size());
  b->max_chunks = max_chunks;

  // device copies: offs (nsys + 1 int64), part_base (nsys int64), items, sys_of (n int32);
  // staged through pinned memory
  const size_t offs_bytes = size_t(2 * nsys + 1) * sizeof(int64_t);
  const size_t items_bytes = std::max<size_t>(1, items.size()) * sizeof(int4);
  const size_t offs_pad = (offs_bytes + 255) / 256 * 256;
  const size_t items_pad = (items_bytes + 255) / 256 * 256;
  const size_t sys_bytes = size_t(std::max<int64_t>(1, b->n)) * sizeof(int);
  int st;
  char *dev = static_cast<char *>(
      workspace(ctx, WS_BATCH, offs_pad + items_pad + sys_bytes, &st));
  if (!dev) return st;
  b->offs = reinterpret_cast<int64_t *>(dev);
  b->part_base = b->offs + nsys + 1;
  b->items = reinterpret_cast<int4 *>(dev + offs_pad);
  b->sys_of = reinterpret_cast<int *>(dev + offs_pad + items_pad);
  const size_t host_bytes = offs_pad + items_pad;
  // the pinned staging buffer may still feed an earlier copy
  RPB_HIP(ctx, hipStreamSynchronize(stream));
  if (ctx->batch_host_bytes < host_bytes) {
    if (ctx->batch_host) RPB_HIP(ctx, hipHostFree(ctx->batch_host));
    ctx->batch_host = nullptr;
    ctx->batch_host_bytes = 0;
    RPB_HIP(ctx, hipHostMalloc(&ctx->batch_host, host_bytes, hipHostMallocDefault));
    ctx->batch_host_bytes = host_bytes;
  }
  char *hb = static_cast<char *>(ctx->batch_host);
  std::memcpy(hb, offs, size_t(nsys + 1) * sizeof(int64_t));
  std::memcpy(hb + size_t(nsys + 1) * sizeof(int64_t), part_base.data(),
              size_t(nsys) * sizeof(int64_t));
  int4 *hi = reinterpret_cast<int4 *>(hb + offs_pad);
  for (size_t q = 0; q < order.size(); ++q) hi[q] = items[order[q]];
  RPB_HIP(ctx, hipMemcpyAsync(b->offs, hb, offs_bytes, hipMemcpyHostToDevice, stream));
  if (!items.empty())
    RPB_HIP(ctx, hipMemcpyAsync(b->items, hi, items.size() * sizeof(int4), hipMemcpyHostToDevice,
                                stream));
  fill_sys_of<<<unsigned(nsys), 256, 0, stream>>>(nsys, b->offs, b->sys_of);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

namespace {

int matvec_batched_sym(rpb_ctx *ctx, const rpb_params *p, const Batch &b, const Packed &g,
                       const void *src, bool has_t, const int *done, int *counter, void *part,
                       const double *h, double *vel, hipStream_t stream) {
  const int64_t n = g.n;
  const bool f64 = g.precision == RPB_FP64;
  const int tpt = b.tpt;
  SymBatchArgs args{b.offs,      b.items, b.nitems, counter, n, int64_t(kBlock) * tpt,
                    b.part_base, done,    done ? done + b.nsys : nullptr, b.nsplit};
  const unsigned grid = unsigned(std::max(1, std::min(b.nitems, b.wgs)));
  double pairs = 0.0;
  for (int s = 0; s < b.nsys; ++s) {
    const double ns = double(b.host_offs[s + 1] - b.host_offs[s]);
    pairs += ns * ns;
  }
  hipEvent_t t0;
  RPB_TRY(timing_begin(ctx, stream, &t0));
  with_variant(has_t, tpt, p->wall != 0, false, [&](auto T, auto P, auto W, auto) {
    constexpr bool kT = decltype(T)::value, kW = decltype(W)::value;
    constexpr int kP = decltype(P)::value;
    if (f64)
      pair_kernel_f64_sym_batched<kP, kT, kW><<<grid, kBlock, 0, stream>>>(
          args, geom_d(g), static_cast<const double *>(src), make_pair_consts<double>(),
          static_cast<double *>(part));
    else
      pair_kernel_mixed_sym_batched<kP, kT, kW><<<grid, kBlock, 0, stream>>>(
          args, geom_f(g), static_cast<const float *>(src), make_pair_consts<float>(),
          static_cast<float *>(part));
  });
  RPB_LAUNCHED(ctx);
  RPB_TRY(timing_end(ctx, stream, t0, pairs, 4 + (f64 ? 0 : 2) + (has_t ? 1 : 0)));
  const double scale = 1.0 / (8.0 * M_PI * p->eta * p->a);
  if (f64)
    reduce_partials_sym_batched<double><<<blocks_for(3 * n, 256), 256, 0, stream>>>(
        args, b.sys_of, static_cast<const double *>(part), h, scale, vel);
  else
    reduce_partials_sym_batched<float><<<blocks_for(3 * n, 256), 256, 0, stream>>>(
        args, b.sys_of, static_cast<const float *>(part), h, scale, vel);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

}  // namespace

int matvec_batched(rpb_ctx *ctx, const rpb_params *p, const Batch &b, const Packed &g,
                   const double *force, const double *torque, const int *done, double *vel,
                   hipStream_t stream) {
  const int64_t n = g.n;
  if (n == 0 || b.nitems == 0) return RPB_OK;
  const bool has_t = torque != nullptr;
  const bool f64 = g.precision == RPB_FP64;
  void *src;
  RPB_TRY(pack_sources(ctx, g, force, torque, &src, stream));
  const double *h = f64 ? geom_d(g).h : geom_f(g).h;
  int st;
  // symmetric items: float32 partials in mixed precision; ordered items: float64
  const size_t part_bytes = b.symmetric
                                ? size_t(b.part_elems) * (f64 ? sizeof(double) : sizeof(float))
                                : size_t(b.max_chunks) * 3 * size_t(n) * sizeof(double);
  void *part = workspace(ctx, WS_PART, std::max<size_t>(8, part_bytes), &st);
  if (!part) return st;
  char *small = static_cast<char *>(workspace(ctx, WS_SMALL, kSmallBytes, &st));
  if (!small) return st;
  int *counter = reinterpret_cast<int *>(small + kSmallWorkCounter);
  zero_int<<<1, 1, 0, stream>>>(counter);
  RPB_LAUNCHED(ctx);
  if (b.symmetric) return matvec_batched_sym(ctx, p, b, g, src, has_t, done, counter, part, h,
                                             vel, stream);

  BatchArgs args{b.offs, b.items, b.nitems, counter, n, b.chunk, done,
                 done ? done + b.nsys : nullptr};
  double *dpart = static_cast<double *>(part);
  const unsigned grid = unsigned(std::max(1, std::min(b.nitems, b.wgs)));
  double pairs = 0.0;
  for (int s = 0; s < b.nsys; ++s) {
    const double ns = double(b.host_offs[s + 1] - b.host_offs[s]);
    pairs += ns * ns;
  }
  hipEvent_t t0;
  RPB_TRY(timing_begin(ctx, stream, &t0));
  const int tpt = b.tpt;
  with_variant(has_t, tpt, p->wall != 0, false, [&](auto T, auto P, auto W, auto) {
    constexpr bool kT = decltype(T)::value, kW = decltype(W)::value;
    constexpr int kP = decltype(P)::value;
    if (f64)
      pair_kernel_f64_batched<kT, kP, kW><<<grid, kBlock, 0, stream>>>(
          args, geom_d(g), static_cast<const double *>(src), make_pair_consts<double>(),
          dpart);
    else
      pair_kernel_mixed_batched<kT, kP, kW><<<grid, kBlock, 0, stream>>>(
          args, geom_f(g), static_cast<const float *>(src), make_pair_consts<float>(), dpart);
  });
  RPB_LAUNCHED(ctx);
  RPB_TRY(timing_end(ctx, stream, t0, pairs, 4 + (f64 ? 0 : 2) + (has_t ? 1 : 0)));
  const double scale = 1.0 / (8.0 * M_PI * p->eta * p->a);
  reduce_partials_batched<<<blocks_for(n, 256), 256, 0, stream>>>(n, b.sys_of, b.offs, b.chunk,
                                                                 done, dpart, h, scale, vel);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

int check_offsets(rpb_ctx *ctx, int32_t nsys, const int64_t *offs) {
  if (nsys < 1) return fail(ctx, RPB_EINVAL, "nsys must be >= 1");
  if (!offs) return fail(ctx, RPB_EINVAL, "offs must not be NULL");
  if (offs[0] != 0) return fail(ctx, RPB_EINVAL, "offs[0] must be 0");
  for (int s = 0; s < nsys; ++s)
    if (offs[s + 1] < offs[s]) return fail(ctx, RPB_EINVAL, "offs must be non-decreasing");
  if (offs[nsys] > (int64_t(1) << 31) - 1)
    return fail(ctx, RPB_EINVAL, "too many spheres for one batch");
  return RPB_OK;
}

}  // namespace rpb

using namespace rpb;

namespace {

int matvec_entry(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                 const double *force, const double *torque, int64_t row0, int64_t row1,
                 double *vel, rpb_stream_t stream_) {
  RPB_TRY(check_params(ctx, p));
  if (n < 0) return fail(ctx, RPB_EINVAL, "n must be >= 0");
  if (row0 < 0 || row1 < row0 || row1 > n)
    return fail(ctx, RPB_EINVAL, "row range [%lld, %lld) outside [0, %lld)", (long long)row0,
                (long long)row1, (long long)n);
  if (n == 0 || row1 == row0) return RPB_OK;
  if (!pos || !vel) return fail(ctx, RPB_EINVAL, "pos and vel_out must not be NULL");
  if (!force && !torque) return fail(ctx, RPB_EINVAL, "force and torque are both NULL");
  const size_t nb = size_t(n) * 3 * sizeof(double);
  const size_t vb = size_t(row1 - row0) * 3 * sizeof(double);
  if (overlaps(vel, vb, pos, nb) || overlaps(vel, vb, force, nb) || overlaps(vel, vb, torque, nb))
    return fail(ctx, RPB_EINVAL, "vel_out overlaps an input");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  RPB_HIP(ctx, hipSetDevice(ctx->device));
  RPB_TRY(check_finite(ctx, pos, n, stream));
  Packed g;
  RPB_TRY(pack_geometry(ctx, p, n, pos, WS_GEOM, &g, stream));
  RPB_TRY(matvec_packed(ctx, p, g, force, torque, row0, row1 - row0, vel, stream));
  return check_output(ctx, vel, 3 * (row1 - row0), stream, "the velocity");
}

}  // namespace

extern "C" {

int rpb_mobility_matvec(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                        const double *force, const double *torque, double *vel_out,
                        rpb_stream_t stream) {
  return matvec_entry(ctx, p, n, pos, force, torque, 0, n, vel_out, stream);
}

int rpb_mobility_matvec_rows(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                             const double *force, const double *torque, int64_t row_begin,
                             int64_t row_end, double *vel_out, rpb_stream_t stream) {
  return matvec_entry(ctx, p, n, pos, force, torque, row_begin, row_end, vel_out, stream);
}

int rpb_mobility_matvec_batched(rpb_ctx *ctx, const rpb_params *p, int32_t nsys,
                                const int64_t *offs, const double *pos, const double *force,
                                const double *torque, double *vel_out, rpb_stream_t stream_) {
  RPB_TRY(check_params(ctx, p));
  RPB_TRY(check_offsets(ctx, nsys, offs));
  if (p->lx > 0.0)
    return fail(ctx, RPB_EINVAL, "pseudo-periodic boundaries are supported for single systems");
  const int64_t n = offs[nsys];
  if (n == 0) return RPB_OK;
  if (!pos || !vel_out) return fail(ctx, RPB_EINVAL, "pos and vel_out must not be NULL");
  if (!force && !torque) return fail(ctx, RPB_EINVAL, "force and torque are both NULL");
  const size_t nb = size_t(n) * 3 * sizeof(double);
  if (overlaps(vel_out, nb, pos, nb) || overlaps(vel_out, nb, force, nb) ||
      overlaps(vel_out, nb, torque, nb))
    return fail(ctx, RPB_EINVAL, "vel_out overlaps an input");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  RPB_HIP(ctx, hipSetDevice(ctx->device));
  RPB_TRY(check_finite(ctx, pos, n, stream));
  Batch b;
  RPB_TRY(prepare_batch(ctx, nsys, offs, p->precision, &b, stream));
  Packed g;
  RPB_TRY(pack_geometry(ctx, p, n, pos, WS_GEOM, &g, stream));
  RPB_TRY(matvec_batched(ctx, p, b, g, force, torque, nullptr, vel_out, stream));
  return check_output(ctx, vel_out, 3 * n, stream, "the velocity");
}

}  // extern "C"
