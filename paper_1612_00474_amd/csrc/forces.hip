// Soft steric forces plus gravity (paper, Sec. III, eq. soft_potential).
//
// U(r) = U0 + U0 (d - r)/b for r < d and U0 exp(-(r - d)/b) for r >= d, with d = 2a and r
// the centre distance for sphere pairs, d = a and r = z for the wall (absent in free space);
// the force is -grad U, magnitude U0/b or (U0/b) exp(-(r - d)/b), repulsive.  Gravity adds
// f_g along z.  Pairs farther than d + 40 b are skipped (their force is below 4.3e-18 U0/b).
// Float64 throughout, unclamped positions, minimum-image separations in a pseudo-periodic box
// (App. B).  Two ways to find the pairs:
//   * cell list (default): spheres binned into cubic cells of side >= d + 40 b, cells hashed
//     to buckets, buckets filled and then sorted by sphere index, each target visiting the 27
//     neighbouring cells in a fixed order: O(N) work, deterministic sums;
//   * all pairs over LDS tiles (a pseudo-periodic box with fewer than three cells per side):
//     the sources split over workgroups and the chunk sums added in a fixed order.
#include <algorithm>
#include <cmath>

#include "rpb_internal.h"

namespace rpb {

namespace {

constexpr int kBlock = 256;
constexpr int kMinWorkgroups = 2048;   // source chunks are added until the grid reaches this

// Sources [s0, s1) against the lane's targets t0 + q kBlock + tid (q < KT) that lie below t1;
// accumulates into f[q][3].  Every lane must call (synchronises).
template <int KT>
__device__ __forceinline__ void steric_accumulate(const double *__restrict__ pos, int64_t t0,
                                                  int64_t t1, int64_t s0, int64_t s1, double a,
                                                  double u0, double b, double lx, double ly,
                                                  double (&f)[KT][3], const double (&tq)[KT][3],
                                                  double *sx, double *sy, double *sz) {
  const int tid = threadIdx.x;
  const double d = 2.0 * a;
  const double cut = d + 40.0 * b;
  const double cut2 = cut * cut;
  const double fmax_ = u0 / b;
  const double inv_b = 1.0 / b;
  for (int64_t j0 = s0; j0 < s1; j0 += kBlock) {
    const int cnt = int(min<int64_t>(kBlock, s1 - j0));
    __syncthreads();
    if (tid < cnt) {
      const int64_t j = j0 + tid;
      sx[tid] = pos[3 * j];
      sy[tid] = pos[3 * j + 1];
      sz[tid] = pos[3 * j + 2];
    }
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      const double xj = sx[jj], yj = sy[jj], zj = sz[jj];
      double dx[KT], dy[KT], dz[KT], r2[KT];
      bool hit = false;
#pragma unroll
      for (int q = 0; q < KT; ++q) {
        dx[q] = tq[q][0] - xj;
        dy[q] = tq[q][1] - yj;
        if (lx > 0.0) {   // pseudo-periodic box: minimum image
          dx[q] -= lx * rint(dx[q] / lx);
          dy[q] -= ly * rint(dy[q] / ly);
        }
        dz[q] = tq[q][2] - zj;
        r2[q] = dx[q] * dx[q] + dy[q] * dy[q] + dz[q] * dz[q];
        hit |= r2[q] < cut2;
      }
      if (hit) {   // rare: a handful of neighbours per target
#pragma unroll
        for (int q = 0; q < KT; ++q) {
          const int64_t i = t0 + q * kBlock + tid;
          if (r2[q] < cut2 && r2[q] > 0.0 && j0 + jj != i && i < t1) {
            const double r = sqrt(r2[q]);
            const double fm = r < d ? fmax_ : fmax_ * exp(-(r - d) * inv_b);
            const double sc = fm / r;
            f[q][0] += sc * dx[q];
            f[q][1] += sc * dy[q];
            f[q][2] += sc * dz[q];
          }
        }
      }
    }
  }
}

// Targets [t0, min(t0 + KT kBlock, t1)) against sources [s0, s1).  FINAL: adds the wall force
// and gravity and stores the force; otherwise stores the pair sum into `out` (a partial).
template <int KT, bool FINAL>
__device__ __forceinline__ void steric_tile(const double *__restrict__ pos, int64_t t0, int64_t t1,
                                            int64_t s0, int64_t s1, double a, double u0, double b,
                                            double lx, double ly, double f_grav_z, int wall,
                                            double *__restrict__ out) {
  __shared__ double sx[kBlock], sy[kBlock], sz[kBlock];
  const int tid = threadIdx.x;
  double f[KT][3], tq[KT][3];
#pragma unroll
  for (int q = 0; q < KT; ++q) {
    const int64_t i = t0 + q * kBlock + tid;
    const int64_t ii = i < t1 ? i : t0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      tq[q][c] = pos[3 * ii + c];
      f[q][c] = 0.0;
    }
  }
  steric_accumulate<KT>(pos, t0, t1, s0, s1, a, u0, b, lx, ly, f, tq, sx, sy, sz);
#pragma unroll
  for (int q = 0; q < KT; ++q) {
    const int64_t i = t0 + q * kBlock + tid;
    if (i < t1) {
      double fz = f[q][2];
      if (FINAL) {
        const double zi = tq[q][2];
        const double fmax_ = u0 / b;
        if (wall) fz += zi < a ? fmax_ : fmax_ * exp(-(zi - a) / b);
        fz += f_grav_z;
      }
      out[3 * i] = f[q][0];
      out[3 * i + 1] = f[q][1];
      out[3 * i + 2] = fz;
    }
  }
}

// grid (target tiles of KT kBlock, source chunks).  One chunk: final forces straight into
// `out`; several: chunk c writes its pair sums to out + 3 n c.
template <int KT, bool FINAL>
__global__ __launch_bounds__(kBlock) void steric_kernel(int64_t n, int64_t chunk,
                                                        const double *__restrict__ pos, double a,
                                                        double u0, double b, double lx, double ly,
                                                        double f_grav_z, int wall,
                                                        double *__restrict__ out) {
  const int64_t t0 = int64_t(blockIdx.x) * kBlock * KT;
  const int64_t s0 = int64_t(blockIdx.y) * chunk;
  const int64_t s1 = min(n, s0 + chunk);
  steric_tile<KT, FINAL>(pos, t0, n, s0, s1, a, u0, b, lx, ly, f_grav_z, wall,
                         out + 3 * n * blockIdx.y);
}

// Sums the chunk partials in chunk order, then adds the wall force and gravity.
__global__ __launch_bounds__(kBlock) void steric_finish(int64_t n, int nchunks,
                                                        const double *__restrict__ pos,
                                                        const double *__restrict__ part, double a,
                                                        double u0, double b, double f_grav_z,
                                                        int wall, double *__restrict__ force) {
  const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;   // element of the (n, 3) array
  if (e >= 3 * n) return;
  double acc = 0.0;
  for (int c = 0; c < nchunks; ++c) acc += part[3 * n * c + e];
  if (e % 3 == 2) {
    const double z = pos[e];
    const double fmax_ = u0 / b;
    if (wall) acc += z < a ? fmax_ : fmax_ * exp(-(z - a) / b);
    acc += f_grav_z;
  }
  force[e] = acc;
}

// ---- cell list ------------------------------------------------------------------------

struct CellArgs {
  double cs;            // cell side along z (and x, y without a box), >= the cutoff
  double csx, csy;      // cell sides along x, y in a box (lx / ncx, ly / ncy)
  double lx, ly;        // box (0: none)
  int ncx, ncy;         // cells per box side (0: none)
  uint32_t mask;        // buckets - 1 (a power of two minus one)
};

__device__ __forceinline__ int clamp_cell(double v) {
  return int(fmin(fmax(floor(v), -1073741824.0), 1073741823.0));
}

// Cell of a position (x, y wrapped into the box when there is one).
__device__ __forceinline__ int3 cell_of(double x, double y, double z, const CellArgs &c) {
  int cx, cy;
  if (c.ncx > 0) {
    const double xw = x - c.lx * floor(x / c.lx), yw = y - c.ly * floor(y / c.ly);
    cx = min(max(clamp_cell(xw / c.csx), 0), c.ncx - 1);
    cy = min(max(clamp_cell(yw / c.csy), 0), c.ncy - 1);
  } else {
    cx = clamp_cell(x / c.cs);
    cy = clamp_cell(y / c.cs);
  }
  return make_int3(cx, cy, clamp_cell(z / c.cs));
}

__device__ __forceinline__ uint32_t bucket_of(int3 q, int sys, uint32_t mask) {
  const uint32_t h = (uint32_t(q.x) * 73856093u) ^ (uint32_t(q.y) * 19349663u) ^
                     (uint32_t(q.z) * 83492791u) ^ (uint32_t(sys) * 2654435761u);
  return h & mask;
}

__global__ void cells_clear(int64_t nb, int *__restrict__ count) {
  const int64_t h = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (h < nb) count[h] = 0;
}

// Cell (and system) of every sphere; bucket occupancy counts.
__global__ void cells_count(int64_t n, const double *__restrict__ pos,
                            const int *__restrict__ sys_of, CellArgs c, int4 *__restrict__ cell,
                            uint32_t *__restrict__ bucket, int *__restrict__ count) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int3 q = cell_of(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], c);
  const int sys = sys_of ? sys_of[i] : 0;
  const uint32_t b = bucket_of(q, sys, c.mask);
  cell[i] = make_int4(q.x, q.y, q.z, sys);
  bucket[i] = b;
  atomicAdd(count + b, 1);
}

// Exclusive prefix sum of the bucket counts into start, in three passes over blocks of kBlock
// buckets (block sums, their scan, then each block's own scan); clears the fill cursors.
__device__ __forceinline__ int block_exclusive_scan(int v, int *tmp) {
  const int tid = threadIdx.x;
  tmp[tid] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const int add = tid >= off ? tmp[tid - off] : 0;
    __syncthreads();
    tmp[tid] += add;
    __syncthreads();
  }
  const int incl = tmp[tid];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kBlock) void cells_block_sums(int64_t nb,
                                                           const int *__restrict__ count,
                                                           int *__restrict__ bsum) {
  __shared__ int tmp[kBlock];
  const int64_t h = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int v = h < nb ? count[h] : 0;
  const int ex = block_exclusive_scan(v, tmp);
  if (threadIdx.x == kBlock - 1) bsum[blockIdx.x] = ex + v;
}

// One workgroup: exclusive scan of the nblk block sums in place (nblk <= kBlock * per).
__global__ __launch_bounds__(kBlock) void cells_scan_sums(int nblk, int *__restrict__ bsum) {
  __shared__ int tmp[kBlock];
  const int per = (nblk + kBlock - 1) / kBlock;
  const int b0 = min(nblk, int(threadIdx.x) * per), b1 = min(nblk, b0 + per);
  int s = 0;
  for (int k = b0; k < b1; ++k) s += bsum[k];
  int run = block_exclusive_scan(s, tmp);
  for (int k = b0; k < b1; ++k) {
    const int v = bsum[k];
    bsum[k] = run;
    run += v;
  }
}

__global__ __launch_bounds__(kBlock) void cells_block_scan(int64_t nb,
                                                           const int *__restrict__ count,
                                                           const int *__restrict__ bsum,
                                                           int *__restrict__ start,
                                                           int *__restrict__ cursor) {
  __shared__ int tmp[kBlock];
  const int64_t h = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int v = h < nb ? count[h] : 0;
  const int ex = block_exclusive_scan(v, tmp);
  if (h < nb) {
    start[h] = bsum[blockIdx.x] + ex;
    cursor[h] = 0;
  }
}

__global__ void cells_fill(int64_t n, const uint32_t *__restrict__ bucket,
                           const int *__restrict__ start, int *__restrict__ cursor,
                           int *__restrict__ list) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t b = bucket[i];
  list[start[b] + atomicAdd(cursor + b, 1)] = int(i);
}

// Sort every bucket's entries by sphere index (heap sort: O(k log k) however full a bucket
// is), so that the order in which a target meets its neighbours depends on the input only.
__global__ void cells_sort(int64_t nb, const int *__restrict__ start, const int *__restrict__ count,
                           int *__restrict__ list) {
  const int64_t h = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (h >= nb) return;
  int *a = list + start[h];
  const int k = count[h];
  if (k < 2) return;
  if (k <= 16) {   // insertion sort for the usual few entries
    for (int u = 1; u < k; ++u) {
      const int v = a[u];
      int w = u - 1;
      while (w >= 0 && a[w] > v) {
        a[w + 1] = a[w];
        --w;
      }
      a[w + 1] = v;
    }
    return;
  }
  auto sift = [a](int root, int end) {
    while (true) {
      int child = 2 * root + 1;
      if (child >= end) return;
      if (child + 1 < end && a[child + 1] > a[child]) ++child;
      if (a[root] >= a[child]) return;
      const int t = a[root];
      a[root] = a[child];
      a[child] = t;
      root = child;
    }
  };
  for (int r = k / 2 - 1; r >= 0; --r) sift(r, k);
  for (int end = k - 1; end > 0; --end) {
    const int t = a[0];
    a[0] = a[end];
    a[end] = t;
    sift(0, end);
  }
}

// Positions and cells in bucket order (sorted slot s holds sphere list[s]), so that a target
// reads each neighbouring bucket as one contiguous range.
__global__ void cells_gather(int64_t n, const int *__restrict__ list,
                             const double *__restrict__ pos, const int4 *__restrict__ cell,
                             double4 *__restrict__ spos, int4 *__restrict__ scell) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int j = list[s];
  spos[s] = make_double4(pos[3 * j], pos[3 * j + 1], pos[3 * j + 2], 0.0);
  int4 q = cell[j];
  q.w = j;   // the system is implied by the bucket check below; keep the index for j != i
  scell[s] = q;
}

// kSterGroup adjacent lanes per target: lane g of the group takes the neighbouring cells
// g, g + kSterGroup, ... of the 27 in a fixed order, each bucket's spheres of that cell (and
// system) in index order; the group's sums are then added by a butterfly over its lanes (a
// fixed order), and its first lane adds the wall force and gravity and writes.  Eight lanes per
// target keep enough wavefronts in flight for small systems (256 spheres: one wavefront per CU
// with one lane per target).
constexpr int kSterGroup = 8;

__global__ void steric_cells(int64_t n, const double *__restrict__ pos, CellArgs c,
                             const int4 *__restrict__ cell, const int *__restrict__ start,
                             const int *__restrict__ count, const double4 *__restrict__ spos,
                             const int4 *__restrict__ scell, const int *__restrict__ sys_of,
                             double a, double u0, double b, double f_grav_z, int wall,
                             double *__restrict__ force) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t i = gid / kSterGroup;
  const int g = int(gid % kSterGroup);
  const bool live = i < n;   // every lane of a group takes part in the butterfly
  const double d = 2.0 * a;
  const double cut = d + 40.0 * b;
  const double cut2 = cut * cut;
  const double fmax_ = u0 / b;
  const double inv_b = 1.0 / b;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  double xi = 0.0, yi = 0.0, zi = 0.0;
  if (live) {
    xi = pos[3 * i];
    yi = pos[3 * i + 1];
    zi = pos[3 * i + 2];
    const int4 me = cell[i];
    for (int o = g; o < 27; o += kSterGroup) {
      const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
      int3 q = make_int3(me.x + ox, me.y + oy, me.z + oz);
      if (c.ncx > 0) {
        q.x = (q.x + c.ncx) % c.ncx;
        q.y = (q.y + c.ncy) % c.ncy;
      }
      const uint32_t h = bucket_of(q, me.w, c.mask);
      const int s0 = start[h], s1 = s0 + count[h];
      for (int s = s0; s < s1; ++s) {
        const int4 cj = scell[s];   // (cell x, y, z, sphere index)
        if (cj.x != q.x || cj.y != q.y || cj.z != q.z || cj.w == i) continue;
        if (sys_of && sys_of[cj.w] != me.w) continue;
        const double4 pj = spos[s];
        double dx = xi - pj.x, dy = yi - pj.y;
        const double dz = zi - pj.z;
        if (c.lx > 0.0) {   // minimum image
          dx -= c.lx * rint(dx / c.lx);
          dy -= c.ly * rint(dy / c.ly);
        }
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < cut2 && r2 > 0.0) {
          const double r = sqrt(r2);
          const double fm = r < d ? fmax_ : fmax_ * exp(-(r - d) * inv_b);
          const double sc = fm / r;
          fx += sc * dx;
          fy += sc * dy;
          fz += sc * dz;
        }
      }
    }
  }
  for (int off = 1; off < kSterGroup; off <<= 1) {
    fx += __shfl_xor(fx, off, kSterGroup);
    fy += __shfl_xor(fy, off, kSterGroup);
    fz += __shfl_xor(fz, off, kSterGroup);
  }
  if (!live || g != 0) return;
  if (wall) fz += zi < a ? fmax_ : fmax_ * exp(-(zi - a) / b);
  fz += f_grav_z;
  force[3 * i] = fx;
  force[3 * i + 1] = fy;
  force[3 * i + 2] = fz;
}

// Cell side and layout for cutoff `cut`; false when a box holds fewer than three cells per
// side (the neighbour cells would then wrap onto each other).
bool cell_args(double cut, double lx, double ly, int64_t n, CellArgs *c) {
  c->cs = cut;
  c->lx = lx;
  c->ly = ly;
  c->ncx = c->ncy = 0;
  c->csx = c->csy = cut;
  if (lx > 0.0) {
    const double nx = std::floor(lx / cut), ny = std::floor(ly / cut);
    if (nx < 3.0 || ny < 3.0) return false;
    c->ncx = int(std::min(nx, 65536.0));
    c->ncy = int(std::min(ny, 65536.0));
    c->csx = lx / c->ncx;
    c->csy = ly / c->ncy;
  }
  uint64_t nb = 1024;
  while (nb < uint64_t(2 * n)) nb <<= 1;
  c->mask = uint32_t(nb - 1);
  return true;
}

// Forces of all spheres (sys_of: sphere -> system map of a batch, NULL for one system).
int steric_cell_run(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                    const int *sys_of, const CellArgs &c, double f_grav_z, double u0, double b,
                    double *force, hipStream_t stream) {
  const int64_t nb = int64_t(c.mask) + 1;
  const size_t cell_bytes = (size_t(n) * sizeof(int4) + 255) / 256 * 256;
  const size_t n_bytes = (size_t(n) * sizeof(int) + 255) / 256 * 256;
  const size_t nb_bytes = (size_t(nb) * sizeof(int) + 255) / 256 * 256;
  int st;
  const int64_t nblk = (nb + kBlock - 1) / kBlock;
  const size_t blk_bytes = (size_t(nblk) * sizeof(int) + 255) / 256 * 256;
  const size_t spos_bytes = (size_t(n) * sizeof(double4) + 255) / 256 * 256;
  char *w = static_cast<char *>(workspace(
      ctx, WS_CELLS, 2 * cell_bytes + spos_bytes + 2 * n_bytes + 3 * nb_bytes + blk_bytes, &st));
  if (!w) return st;
  int4 *cell = reinterpret_cast<int4 *>(w);
  uint32_t *bucket = reinterpret_cast<uint32_t *>(w + cell_bytes);
  int *list = reinterpret_cast<int *>(w + cell_bytes + n_bytes);
  int *count = reinterpret_cast<int *>(w + cell_bytes + 2 * n_bytes);
  int *start = count + nb_bytes / sizeof(int);
  int *cursor = start + nb_bytes / sizeof(int);
  int *bsum = cursor + nb_bytes / sizeof(int);
  char *tail = reinterpret_cast<char *>(bsum) + blk_bytes;
  int4 *scell = reinterpret_cast<int4 *>(tail);
  double4 *spos = reinterpret_cast<double4 *>(tail + cell_bytes);
  const unsigned gn = unsigned((n + kBlock - 1) / kBlock), gb = unsigned((nb + kBlock - 1) / kBlock);
  cells_clear<<<gb, kBlock, 0, stream>>>(nb, count);
  RPB_LAUNCHED(ctx);
  cells_count<<<gn, kBlock, 0, stream>>>(n, pos, sys_of, c, cell, bucket, count);
  RPB_LAUNCHED(ctx);
  cells_block_sums<<<gb, kBlock, 0, stream>>>(nb, count, bsum);
  RPB_LAUNCHED(ctx);
  cells_scan_sums<<<1, kBlock, 0, stream>>>(int(gb), bsum);
  RPB_LAUNCHED(ctx);
  cells_block_scan<<<gb, kBlock, 0, stream>>>(nb, count, bsum, start, cursor);
  RPB_LAUNCHED(ctx);
  cells_fill<<<gn, kBlock, 0, stream>>>(n, bucket, start, cursor, list);
  RPB_LAUNCHED(ctx);
  cells_sort<<<gb, kBlock, 0, stream>>>(nb, start, count, list);
  RPB_LAUNCHED(ctx);
  cells_gather<<<gn, kBlock, 0, stream>>>(n, list, pos, cell, spos, scell);
  RPB_LAUNCHED(ctx);
  steric_cells<<<unsigned((n * kSterGroup + kBlock - 1) / kBlock), kBlock, 0, stream>>>(
      n, pos, c, cell, start, count, spos, scell, sys_of, p->a, u0, b, f_grav_z, p->wall, force);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

}  // namespace

int forces_batched_run(rpb_ctx *ctx, const rpb_params *p, const Batch &bt, const double *pos,
                       double f_grav_z, double u0, double b, double *force, hipStream_t stream) {
  if (bt.n <= 0) return RPB_OK;
  CellArgs c;
  cell_args(2.0 * p->a + 40.0 * b, 0.0, 0.0, bt.n, &c);
  return steric_cell_run(ctx, p, bt.n, pos, bt.sys_of, c, f_grav_z, u0, b, force, stream);
}

int forces_run(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos, double f_grav_z,
               double u0, double b, double *force, hipStream_t stream) {
  if (n <= 0) return RPB_OK;
  const double cut = 2.0 * p->a + 40.0 * b;
  if (p->lx > 0.0 && (p->lx <= 2.0 * cut || p->ly <= 2.0 * cut))
    return fail(ctx, RPB_EINVAL, "box %g x %g too small for the minimum image (need > %g)", p->lx,
                p->ly, 2.0 * cut);
  CellArgs c;
  if (cell_args(cut, p->lx, p->ly, n, &c))
    return steric_cell_run(ctx, p, n, pos, nullptr, c, f_grav_z, u0, b, force, stream);
  // a box with fewer than three cells per side: all pairs
  constexpr int kTargets = 2;
  const int64_t per = int64_t(kBlock) * kTargets;
  const int64_t tiles = (n + per - 1) / per;
  // split the sources (in whole LDS tiles) until the grid fills the chip
  const int64_t ltiles = (n + kBlock - 1) / kBlock;
  const int64_t want = std::min<int64_t>({(kMinWorkgroups + tiles - 1) / tiles, ltiles, 64});
  const int64_t chunk = (ltiles + want - 1) / want * kBlock;
  const int64_t nchunks = (n + chunk - 1) / chunk;
  if (tiles > 0x7fffffff) return fail(ctx, RPB_EINVAL, "too many spheres");
  if (nchunks == 1) {
    steric_kernel<kTargets, true><<<dim3{unsigned(tiles), 1u, 1u}, kBlock, 0, stream>>>(
        n, chunk, pos, p->a, u0, b, p->lx, p->ly, f_grav_z, p->wall, force);
    RPB_LAUNCHED(ctx);
    return RPB_OK;
  }
  int st;
  double *part = static_cast<double *>(
      workspace(ctx, WS_PART, size_t(nchunks) * 3 * size_t(n) * sizeof(double), &st));
  if (!part) return st;
  steric_kernel<kTargets, false><<<dim3{unsigned(tiles), unsigned(nchunks), 1u}, kBlock, 0,
                                   stream>>>(n, chunk, pos, p->a, u0, b, p->lx, p->ly, f_grav_z,
                                             p->wall, part);
  RPB_LAUNCHED(ctx);
  const int64_t elems = 3 * n;
  steric_finish<<<unsigned((elems + kBlock - 1) / kBlock), kBlock, 0, stream>>>(
      n, int(nchunks), pos, part, p->a, u0, b, f_grav_z, p->wall, force);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

}  // namespace rpb

using namespace rpb;

extern "C" int rpb_forces(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                          double f_grav_z, double u0, double b, double *force_out,
                          rpb_stream_t stream_) {
  RPB_TRY(check_params(ctx, p));
  if (n < 0) return fail(ctx, RPB_EINVAL, "n must be >= 0");
  if (!(u0 >= 0.0) || !(b > 0.0)) return fail(ctx, RPB_EINVAL, "need u0 >= 0 and b > 0");
  if (n == 0) return RPB_OK;
  if (!pos || !force_out) return fail(ctx, RPB_EINVAL, "pos and force_out must not be NULL");
  const size_t nb = size_t(n) * 3 * sizeof(double);
  if (overlaps(force_out, nb, pos, nb)) return fail(ctx, RPB_EINVAL, "force_out overlaps pos");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  RPB_HIP(ctx, hipSetDevice(ctx->device));
  RPB_TRY(check_finite(ctx, pos, n, stream));
  return forces_run(ctx, p, n, pos, f_grav_z, u0, b, force_out, stream);
}
