// Matrix-free product U = M F + M_C T of the regularised Rotne-Prager-Blake mobility.
//
// Direct summation over all ordered pairs (paper, Sec. II.B): the pair tensor is evaluated
// on the fly (pair_tensor.h) and never stored, so the kernel is bound by the vector ALUs,
// not by HBM.  Layout:
//   pack_geometry   O(N)   AoS float64 positions -> SoA clamped heights, weights H0(z/a)
//                          (App. A, eq. effMob); mixed precision splits x, y into
//                          float32 hi + lo so that near-pair separations keep ~1e-7 accuracy
//                          far from the origin.
//   pack_vectors    O(N)   AoS float64 force/torque -> SoA H-weighted source vectors.
//   pair_kernel     O(N^2) grid (target tile, source chunk); each workgroup stages source
//                          tiles in LDS and every lane accumulates one target; float64
//                          sums, or float32 sums with Kahan compensation.
//   reduce_partials O(N S) fixed-order sum over source chunks, times H_i / (8 pi eta).
#include <algorithm>
#include <cmath>

#include "pair_tensor.h"
#include "rpb_internal.h"

namespace rpb {

namespace {

constexpr int kBlock = 256;           // lanes per workgroup = targets per tile = sources per LDS tile

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

__global__ void pack_geometry_f64(int64_t n, const double *__restrict__ pos, double a,
                                  double *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double z = pos[3 * i + 2];
  out[i] = pos[3 * i];
  out[n + i] = pos[3 * i + 1];
  out[2 * n + i] = fmax(z, a);
  out[3 * n + i] = fmin(fmax(z / a, 0.0), 1.0);
}

__global__ void pack_geometry_mixed(int64_t n, const double *__restrict__ pos, double a,
                                    double *__restrict__ hout, float *__restrict__ f) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
  const float xh = float(x), yh = float(y);
  f[i] = xh;
  f[n + i] = float(x - double(xh));
  f[2 * n + i] = yh;
  f[3 * n + i] = float(y - double(yh));
  f[4 * n + i] = float(fmax(z, a));
  hout[i] = fmin(fmax(z / a, 0.0), 1.0);
}

// Source vectors, H-weighted, structure of arrays: [fx | fy | fz | tx | ty | tz] (n each).
template <typename Real>
__global__ void pack_vectors(int64_t n, const double *__restrict__ h,
                             const double *__restrict__ force, const double *__restrict__ torque,
                             Real *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double w = h[i];
  for (int c = 0; c < 3; ++c) {
    out[c * n + i] = force ? Real(w * force[3 * i + c]) : Real(0);
    if (torque) out[(3 + c) * n + i] = Real(w * torque[3 * i + c]);
  }
}

struct PairArgs {
  int64_t n;        // sources (and geometry size)
  int64_t row0;     // first target
  int64_t nrows;    // number of targets
  int64_t chunk;    // sources per workgroup (multiple of kBlock)
};

__device__ __forceinline__ void kahan_add(float &s, float &c, float v) {
  const float y = v - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}

// float64 pair kernel.  Workgroup = kBlock lanes x TPT targets per lane; the source chunk
// blockIdx.y is streamed through LDS in tiles of kBlock.  Output:
// partial[(chunk * 3 + comp) * nrows + row].
template <bool TORQUE, int TPT>
__global__ __launch_bounds__(kBlock) void pair_kernel_f64(PairArgs args, GeomD g,
                                                          const double *__restrict__ src,
                                                          PairConsts<double> k,
                                                          double *__restrict__ partial) {
  __shared__ double sx[kBlock], sy[kBlock], sz[kBlock];
  __shared__ double sf[3][kBlock];
  __shared__ double st[TORQUE ? 3 : 1][kBlock];

  const int tid = threadIdx.x;
  const int64_t n = args.n;
  int64_t r[TPT];
  double xi[TPT], yi[TPT], zi[TPT], u[TPT][3];
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    r[q] = int64_t(blockIdx.x) * (kBlock * TPT) + q * kBlock + tid;
    const int64_t i = args.row0 + (r[q] < args.nrows ? r[q] : 0);
    xi[q] = g.x[i];
    yi[q] = g.y[i];
    zi[q] = g.z[i];
    u[q][0] = u[q][1] = u[q][2] = 0.0;
  }
  const int64_t jb = int64_t(blockIdx.y) * args.chunk;
  const int64_t je = min(n, jb + args.chunk);

  for (int64_t t0 = jb; t0 < je; t0 += kBlock) {
    const int cnt = int(min<int64_t>(kBlock, je - t0));
    __syncthreads();
    if (tid < cnt) {
      const int64_t j = t0 + tid;
      sx[tid] = g.x[j];
      sy[tid] = g.y[j];
      sz[tid] = g.z[j];
      sf[0][tid] = src[j];
      sf[1][tid] = src[n + j];
      sf[2][tid] = src[2 * n + j];
      if (TORQUE) {
        st[0][tid] = src[3 * n + j];
        st[1][tid] = src[4 * n + j];
        st[2][tid] = src[5 * n + j];
      }
    }
    __syncthreads();
#pragma unroll 2
    for (int j = 0; j < cnt; ++j) {
      const double xj = sx[j], yj = sy[j], zj = sz[j];
      const double fx = sf[0][j], fy = sf[1][j], fz = sf[2][j];
      const double tx = TORQUE ? st[0][j] : 0.0, ty = TORQUE ? st[1][j] : 0.0,
                   tz = TORQUE ? st[2][j] : 0.0;
#pragma unroll
      for (int q = 0; q < TPT; ++q) {
        double ox, oy, oz;
        pair_velocity<double, TORQUE>(xi[q] - xj, yi[q] - yj, zi[q], zj, fx, fy, fz, tx, ty, tz,
                                      k, ox, oy, oz);
        u[q][0] += ox;
        u[q][1] += oy;
        u[q][2] += oz;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    if (r[q] < args.nrows) {
      const int64_t base = int64_t(blockIdx.y) * 3 * args.nrows + r[q];
      partial[base] = u[q][0];
      partial[base + args.nrows] = u[q][1];
      partial[base + 2 * args.nrows] = u[q][2];
    }
  }
}

// Mixed pair kernel: float32 pair terms, float32 sums over each LDS tile of kBlock sources,
// tile sums added with Kahan compensation per target, float64 partials.
template <bool TORQUE, int TPT>
__global__ __launch_bounds__(kBlock) void pair_kernel_mixed(PairArgs args, GeomF g,
                                                            const float *__restrict__ src,
                                                            PairConsts<float> k,
                                                            double *__restrict__ partial) {
  __shared__ float sxh[kBlock], sxl[kBlock], syh[kBlock], syl[kBlock], sz[kBlock];
  __shared__ float sf[3][kBlock];
  __shared__ float st[TORQUE ? 3 : 1][kBlock];

  const int tid = threadIdx.x;
  const int64_t n = args.n;
  int64_t r[TPT];
  float xih[TPT], xil[TPT], yih[TPT], yil[TPT], zi[TPT];
  float s[TPT][3], c[TPT][3];
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    r[q] = int64_t(blockIdx.x) * (kBlock * TPT) + q * kBlock + tid;
    const int64_t i = args.row0 + (r[q] < args.nrows ? r[q] : 0);
    xih[q] = g.xh[i];
    xil[q] = g.xl[i];
    yih[q] = g.yh[i];
    yil[q] = g.yl[i];
    zi[q] = g.z[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) s[q][d] = c[q][d] = 0.f;
  }
  const int64_t jb = int64_t(blockIdx.y) * args.chunk;
  const int64_t je = min(n, jb + args.chunk);

  for (int64_t t0 = jb; t0 < je; t0 += kBlock) {
    const int cnt = int(min<int64_t>(kBlock, je - t0));
    __syncthreads();
    if (tid < cnt) {
      const int64_t j = t0 + tid;
      sxh[tid] = g.xh[j];
      sxl[tid] = g.xl[j];
      syh[tid] = g.yh[j];
      syl[tid] = g.yl[j];
      sz[tid] = g.z[j];
      sf[0][tid] = src[j];
      sf[1][tid] = src[n + j];
      sf[2][tid] = src[2 * n + j];
      if (TORQUE) {
        st[0][tid] = src[3 * n + j];
        st[1][tid] = src[4 * n + j];
        st[2][tid] = src[5 * n + j];
      }
    }
    __syncthreads();
    float a[TPT][3];
#pragma unroll
    for (int q = 0; q < TPT; ++q) a[q][0] = a[q][1] = a[q][2] = 0.f;
#pragma unroll 2
    for (int j = 0; j < cnt; ++j) {
      const float xjh = sxh[j], xjl = sxl[j], yjh = syh[j], yjl = syl[j], zj = sz[j];
      const float fx = sf[0][j], fy = sf[1][j], fz = sf[2][j];
      const float tx = TORQUE ? st[0][j] : 0.f, ty = TORQUE ? st[1][j] : 0.f,
                  tz = TORQUE ? st[2][j] : 0.f;
#pragma unroll
      for (int q = 0; q < TPT; ++q) {
        const float dx = (xih[q] - xjh) + (xil[q] - xjl);
        const float dy = (yih[q] - yjh) + (yil[q] - yjl);
        float ox, oy, oz;
        pair_velocity<float, TORQUE>(dx, dy, zi[q], zj, fx, fy, fz, tx, ty, tz, k, ox, oy, oz);
        a[q][0] += ox;
        a[q][1] += oy;
        a[q][2] += oz;
      }
    }
#pragma unroll
    for (int q = 0; q < TPT; ++q)
#pragma unroll
      for (int d = 0; d < 3; ++d) kahan_add(s[q][d], c[q][d], a[q][d]);
  }
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    if (r[q] < args.nrows) {
      const int64_t base = int64_t(blockIdx.y) * 3 * args.nrows + r[q];
      partial[base] = double(s[q][0]) - double(c[q][0]);
      partial[base + args.nrows] = double(s[q][1]) - double(c[q][1]);
      partial[base + 2 * args.nrows] = double(s[q][2]) - double(c[q][2]);
    }
  }
}

__global__ void reduce_partials(int64_t nrows, int nchunks, const double *__restrict__ partial,
                                const double *__restrict__ h, double scale,
                                double *__restrict__ vel) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const double w = scale * h[r];
  for (int c = 0; c < 3; ++c) {
    double s = 0.0;
    for (int q = 0; q < nchunks; ++q) s += partial[(int64_t(q) * 3 + c) * nrows + r];
    vel[3 * r + c] = w * s;
  }
}

__global__ void finite_flag(int64_t m, const double *__restrict__ v, int *__restrict__ flag) {
  int bad = 0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < m;
       i += int64_t(gridDim.x) * blockDim.x)
    bad |= !isfinite(v[i]);
  if (bad) flag[0] = 1;   // benign race: every writer stores the same value
}

__global__ void zero_int(int *p) { p[0] = 0; }

inline unsigned blocks_for(int64_t n, int threads) {
  return unsigned((n + threads - 1) / threads);
}

}  // namespace

int check_finite(rpb_ctx *ctx, const double *pos, int64_t n, hipStream_t stream) {
  int st;
  int *flag = static_cast<int *>(workspace(ctx, WS_SMALL, 1 << 16, &st));
  if (!flag) return st;
  int *f = flag + (1 << 14) - 1;  // last int of the small slot's first 64 KiB
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

int pack_geometry(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos, Slot slot,
                  Packed *out, hipStream_t stream) {
  int st;
  void *buf = workspace(ctx, slot, geom_bytes(n, p->precision), &st);
  if (!buf) return st;
  out->n = n;
  out->precision = p->precision;
  out->geom = buf;
  if (p->precision == RPB_FP64) {
    pack_geometry_f64<<<blocks_for(n, 256), 256, 0, stream>>>(n, pos, p->a,
                                                              static_cast<double *>(buf));
  } else {
    double *h = static_cast<double *>(buf);
    pack_geometry_mixed<<<blocks_for(n, 256), 256, 0, stream>>>(
        n, pos, p->a, h, reinterpret_cast<float *>(h + n));
  }
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

int matvec_packed(rpb_ctx *ctx, const rpb_params *p, const Packed &g, const double *force,
                  const double *torque, int64_t row0, int64_t nrows, double *vel,
                  hipStream_t stream) {
  const int64_t n = g.n;
  if (nrows <= 0) return RPB_OK;
  const bool has_t = torque != nullptr;
  const bool f64 = g.precision == RPB_FP64;
  const size_t esz = f64 ? sizeof(double) : sizeof(float);
  int st;
  void *src = workspace(ctx, WS_SRC, size_t(6 * n) * esz, &st);
  if (!src) return st;
  const double *h = f64 ? geom_d(g).h : geom_f(g).h;
  if (f64)
    pack_vectors<double><<<blocks_for(n, 256), 256, 0, stream>>>(n, h, force, torque,
                                                                 static_cast<double *>(src));
  else
    pack_vectors<float><<<blocks_for(n, 256), 256, 0, stream>>>(n, h, force, torque,
                                                                static_cast<float *>(src));
  RPB_LAUNCHED(ctx);

  // Source chunking: enough workgroups to fill the chip several times over.  The chunks
  // depend on n only (not on the row range), so every target sums its sources in the same
  // order whichever rows are requested: row shards concatenate to the full product bitwise.
  const int tpt = f64 ? ctx->tune.tpt_f64 : ctx->tune.tpt_mixed;
  const int64_t per_wg = int64_t(kBlock) * tpt;
  const int64_t tiles = (nrows + per_wg - 1) / per_wg;
  const int64_t tiles_full = (n + per_wg - 1) / per_wg;
  int64_t nchunks =
      std::max<int64_t>(1, (int64_t(ctx->tune.target_wgs) + tiles_full - 1) / tiles_full);
  int64_t chunk = (n + nchunks - 1) / nchunks;
  chunk = std::max<int64_t>(kBlock, (chunk + kBlock - 1) / kBlock * kBlock);
  nchunks = (n + chunk - 1) / chunk;
  if (tiles > 0x7fffffff || nchunks > 65535)
    return fail(ctx, RPB_EINVAL, "problem too large for one launch (n = %lld)", (long long)n);

  double *part = static_cast<double *>(
      workspace(ctx, WS_PART, size_t(nchunks) * 3 * size_t(nrows) * sizeof(double), &st));
  if (!part) return st;

  PairArgs args{n, row0, nrows, chunk};
  const dim3 grid{unsigned(tiles), unsigned(nchunks), 1u};
  hipEvent_t t0;
  RPB_TRY(timing_begin(ctx, stream, &t0));
  if (f64) {
    const auto k = make_pair_consts<double>(p->a);
    const double *sv = static_cast<const double *>(src);
    const GeomD gd = geom_d(g);
    if (has_t && tpt == 2)
      pair_kernel_f64<true, 2><<<grid, kBlock, 0, stream>>>(args, gd, sv, k, part);
    else if (has_t)
      pair_kernel_f64<true, 1><<<grid, kBlock, 0, stream>>>(args, gd, sv, k, part);
    else if (tpt == 2)
      pair_kernel_f64<false, 2><<<grid, kBlock, 0, stream>>>(args, gd, sv, k, part);
    else
      pair_kernel_f64<false, 1><<<grid, kBlock, 0, stream>>>(args, gd, sv, k, part);
  } else {
    const auto k = make_pair_consts<float>(p->a);
    const float *sv = static_cast<const float *>(src);
    const GeomF gf = geom_f(g);
    if (has_t && tpt == 2)
      pair_kernel_mixed<true, 2><<<grid, kBlock, 0, stream>>>(args, gf, sv, k, part);
    else if (has_t)
      pair_kernel_mixed<true, 1><<<grid, kBlock, 0, stream>>>(args, gf, sv, k, part);
    else if (tpt == 2)
      pair_kernel_mixed<false, 2><<<grid, kBlock, 0, stream>>>(args, gf, sv, k, part);
    else
      pair_kernel_mixed<false, 1><<<grid, kBlock, 0, stream>>>(args, gf, sv, k, part);
  }
  RPB_LAUNCHED(ctx);
  RPB_TRY(timing_end(ctx, stream, t0, double(nrows) * double(n),
                     (f64 ? 0 : 2) + (has_t ? 1 : 0)));

  const double scale = 1.0 / (8.0 * M_PI * p->eta);
  reduce_partials<<<blocks_for(nrows, 256), 256, 0, stream>>>(nrows, int(nchunks), part,
                                                              h + row0, scale, vel);
  RPB_LAUNCHED(ctx);
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
  return matvec_packed(ctx, p, g, force, torque, row0, row1 - row0, vel, stream);
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

}  // extern "C"
