// Weights, y-weighted density channels and mass assignment (Sec. 4.1, eq. 34;
// Sec. 4.2, eq. 39; Sec. 5.2, eq. 53).
//
// Assignment is a gather over tiles: particles are bucketed by the T^3 tile of
// their cell, and one workgroup per output tile scatters the particles of the
// 27 neighbouring tiles into LDS. Contributions are rounded to 64-bit fixed
// point (scale 2^e with sum|w| 2^e < 2^61) and added with integer LDS atomics,
// so every grid value is independent of thread and bucket order: the result is
// bitwise reproducible.
#include <cmath>

#include "tsb_internal.h"

namespace tsb {

namespace {

constexpr int kMaxCh = 48;       // real channels (+1 randoms channel in survey mode)
constexpr int kMaxGrids = 32;
constexpr int kPrepBlocks = 512;
constexpr int kDenseMin = 8;     // particles sharing a (cell, half-cell octant) that go by moments
constexpr int kMaxDense = 64;    // moment groups per tile (further groups stay on the direct path)

struct CatPtrs {
  const float *x, *y, *z, *w, *nbar;
  int64_t n;
};

CatPtrs cat_ptrs(const tsb_catalog* c) {
  CatPtrs p{};
  if (c) {
    p.x = c->x; p.y = c->y; p.z = c->z; p.w = c->w; p.nbar = c->nbar; p.n = c->n;
  }
  return p;
}

__device__ inline double particle_weight(const CatPtrs& c, int64_t i, double P0) {
  double w = c.w ? (double)c.w[i] : 1.0;
  if (c.nbar && P0 > 0.0) w = w / (1.0 + (double)c.nbar[i] * P0);
  return w;
}

// ----------------------------------------------------------------------------
// weights: sums, alpha, fixed-point scale, input validation

struct PrepArgs {
  CatPtrs d, r;
  double P0, inv_h, origin[3], obs[3];
  int N, box_mode, local;
  DevScalars* scal;
  double* partials;   // [gridDim][4]
};

__device__ inline void block_sum4(double* v, double* sh) {
  // fixed-order tree over the block
  const int t = threadIdx.x;
  for (int k = 0; k < 4; ++k) sh[k * kBlock + t] = v[k];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (t < s)
      for (int k = 0; k < 4; ++k) sh[k * kBlock + t] += sh[k * kBlock + t + s];
    __syncthreads();
  }
  for (int k = 0; k < 4; ++k) v[k] = sh[k * kBlock];
}

__global__ void __launch_bounds__(kBlock) prep_kernel(PrepArgs a) {
  __shared__ double sh[4 * kBlock];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  int err = 0;
  const int64_t ntot = a.d.n + a.r.n;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < ntot;
       i += (int64_t)gridDim.x * kBlock) {
    const bool ran = i >= a.d.n;
    const CatPtrs& c = ran ? a.r : a.d;
    const int64_t j = ran ? i - a.d.n : i;
    const double x = c.x[j], y = c.y[j], z = c.z[j];
    const double w = particle_weight(c, j, a.P0);
    if (!isfinite(x) || !isfinite(y) || !isfinite(z) || !isfinite(w)) {
      err |= 1;
      continue;
    }
    if (!a.box_mode) {
      const double ux = (x - a.origin[0]) * a.inv_h, uy = (y - a.origin[1]) * a.inv_h,
                   uz = (z - a.origin[2]) * a.inv_h;
      if (ux < 0.0 || ux >= a.N || uy < 0.0 || uy >= a.N || uz < 0.0 || uz >= a.N) err |= 2;
    }
    if (a.local && x == a.obs[0] && y == a.obs[1] && z == a.obs[2]) err |= 4;
    if (ran) {
      v[1] += w;
      v[3] += fabs(w);
    } else {
      v[0] += w;
      v[2] += fabs(w);
    }
  }
  if (err) atomicOr(&a.scal->err, err);
  block_sum4(v, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) a.partials[blockIdx.x * 4 + k] = v[k];
}

__global__ void __launch_bounds__(kBlock) prep_final_kernel(const double* partials, int nblocks,
                                                            DevScalars* scal, int box_mode,
                                                            double n3, double volume) {
  __shared__ double sh[4 * kBlock];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += kBlock)
    for (int k = 0; k < 4; ++k) v[k] += partials[b * 4 + k];
  block_sum4(v, sh);
  if (threadIdx.x == 0) {
    scal->sum_w = v[0];
    scal->sum_w_ran = v[1];
    scal->sum_abs = v[2];
    scal->sum_abs_ran = v[3];
    const double alpha = box_mode ? 0.0 : (v[1] != 0.0 ? v[0] / v[1] : 0.0);   // Sec. 4.1
    scal->alpha = alpha;
    const double wtot = v[2] + fabs(alpha) * v[3];
    int e = 40;
    if (wtot > 0.0 && isfinite(wtot)) {
      int ex;
      frexp(wtot, &ex);   // wtot < 2^ex
      e = 61 - ex;
      if (e > 200) e = 200;
      if (e < -200) e = -200;
    }
    scal->scale = ldexp(1.0, e);
    scal->inv_scale = ldexp(1.0, -e);
    scal->mean_cell = box_mode ? v[0] / n3 : 0.0;
    scal->I = box_mode ? v[0] * v[0] * v[0] / (volume * volume) : 0.0;   // Sec. 4.4
  }
}

// ----------------------------------------------------------------------------
// bucketing by tile

struct BucketArgs {
  CatPtrs d, r;
  double inv_h, origin[3];
  int N, T, NT;
  int* count;
  int* cursor;
  const int* start;
  int* keys;
};

__device__ inline int cell_of(double u, int N) {
  // cell index of a grid coordinate, taken periodically; non-finite -> 0
  if (!isfinite(u)) return 0;
  double c = floor(u);
  c = c - (double)N * floor(c / (double)N);
  int i = (int)c;
  return i < 0 ? 0 : (i >= N ? N - 1 : i);
}

__global__ void __launch_bounds__(kBlock) bucket_count_kernel(BucketArgs a) {
  const int64_t ntot = a.d.n + a.r.n;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < ntot;
       i += (int64_t)gridDim.x * kBlock) {
    const bool ran = i >= a.d.n;
    const CatPtrs& c = ran ? a.r : a.d;
    const int64_t j = ran ? i - a.d.n : i;
    const int cx = cell_of(((double)c.x[j] - a.origin[0]) * a.inv_h, a.N);
    const int cy = cell_of(((double)c.y[j] - a.origin[1]) * a.inv_h, a.N);
    const int cz = cell_of(((double)c.z[j] - a.origin[2]) * a.inv_h, a.N);
    const int key = ((cx / a.T) * a.NT + cy / a.T) * a.NT + cz / a.T;
    a.keys[i] = key;
    atomicAdd(&a.count[key], 1);
  }
}

// exclusive prefix sum of n ints by one workgroup (n <= 2^21)
__global__ void __launch_bounds__(1024) scan_kernel(const int* in, int* out, int n) {
  __shared__ int sh[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int b0 = t * per, b1 = min(n, b0 + per);
  int s = 0;
  for (int i = b0; i < b1; ++i) s += in[i];
  sh[t] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan of the 1024 chunk sums
  for (int off = 1; off < 1024; off <<= 1) {
    int v = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  int run = sh[t] - s;
  for (int i = b0; i < b1; ++i) {
    out[i] = run;
    run += in[i];
  }
}

// Channel layout shared by the record and tile kernels.
struct ChanInfo {
  int nch;                     // real channels (the survey randoms channel is nch)
  int local;
  double obs[3];
  int chL[kMaxCh], chM[kMaxCh], chPart[kMaxCh];
  double ynorm[45];
};

template <int NCH>
__device__ inline void channel_values(const ChanInfo& ci, double x, double y, double z, double w, bool ran,
                                      double alpha, double* cv) {
  // c = w y_L^M*(x^) (eq. 34); randoms carry -alpha (eq. 34); survey mode adds
  // the randoms channel (weight w, randoms only) used by the normalisation
  double ux = 0.0, uy = 0.0, uz = 1.0;
  if (ci.local) {
    const double dx = x - ci.obs[0], dy = y - ci.obs[1], dz = z - ci.obs[2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (r > 0.0) {
      ux = dx / r;
      uy = dy / r;
      uz = dz / r;
    }
  }
  const double s = ran ? -alpha * w : w;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    if (c >= ci.nch) {
      cv[c] = (c == ci.nch && ran) ? w : 0.0;
      continue;
    }
    double re = 1.0, im = 0.0;
    if (ci.local) ylm_pos_m(ci.chL[c], ci.chM[c], ux, uy, uz, ci.ynorm, &re, &im);
    // Re(y*) = Re(y), Im(y*) = -Im(y)
    cv[c] = s * (ci.chPart[c] ? -im : re);
  }
}

// Particle records in bucket order: grid coordinate u (FP64; NaN marks a
// particle that takes no part) and its channel weights.
template <typename T>
struct Records {
  double* ux;
  double* uy;
  double* uz;
  T* cv;                       // [nchx][cap]
  int64_t cap;
};

template <typename T, int NCH>
struct FillArgs {
  BucketArgs b;
  ChanInfo ci;
  Records<T> rec;
  double P0;
  int box_mode, nchx;
  const DevScalars* scal;
};

template <typename T, int NCH>
__global__ void __launch_bounds__(kBlock) bucket_fill_kernel(FillArgs<T, NCH> a) {
  const int64_t ntot = a.b.d.n + a.b.r.n;
  const double alpha = a.scal->alpha;
  const int N = a.b.N;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < ntot;
       i += (int64_t)gridDim.x * kBlock) {
    const int key = a.b.keys[i];
    const int slot = a.b.start[key] + atomicAdd(&a.b.cursor[key], 1);
    const bool ran = i >= a.b.d.n;
    const CatPtrs& c = ran ? a.b.r : a.b.d;
    const int64_t j = ran ? i - a.b.d.n : i;
    const double x = c.x[j], y = c.y[j], z = c.z[j];
    const double w = particle_weight(c, j, a.P0);
    double u[3] = {(x - a.b.origin[0]) * a.b.inv_h, (y - a.b.origin[1]) * a.b.inv_h,
                   (z - a.b.origin[2]) * a.b.inv_h};
    bool ok = isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]) && isfinite(w);
    for (int ax = 0; ax < 3 && ok; ++ax) {
      if (u[ax] < 0.0 || u[ax] >= N) {
        if (!a.box_mode) ok = false;   // reported by the weight pass
        else u[ax] -= N * floor(u[ax] / N);
      }
    }
    a.rec.ux[slot] = ok ? u[0] : NAN;
    a.rec.uy[slot] = u[1];
    a.rec.uz[slot] = u[2];
    double cv[NCH];
    channel_values<NCH>(a.ci, x, y, z, ok ? w : 0.0, ran, alpha, cv);
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
      if (ch < a.nchx) a.rec.cv[(int64_t)ch * a.rec.cap + slot] = (T)cv[ch];
  }
}

// ----------------------------------------------------------------------------
// dense groups: particles of one cell and one half-cell octant share the
// stencil nodes of both interlaced grids, and their order-p weights are
// polynomials (degree <= 2) in the in-cell offset f = u - floor(u). Such a
// group is reduced once to the moments sum_i c_i f_x^a f_y^b f_z^c (a,b,c <= 2,
// 64-bit fixed point, order-independent) and its node contributions follow
// from the moments. This removes the serialised LDS atomics of crowded cells.

struct GroupDesc { int start, count, key, pad; };

// Key (local cell * 8 + octant) of a record in the tile at (ox, oy, oz), or -1
// when the record is invalid or its stencils are not the group's canonical
// ones (then it stays on the direct path).
__device__ inline int group_key(const double* u, const int* o, int T, int p, int copies) {
  if (!isfinite(u[0]) || !isfinite(u[1]) || !isfinite(u[2])) return -1;
  int cell = 0, oct = 0;
  for (int ax = 0; ax < 3; ++ax) {
    const double c = floor(u[ax]);
    const int bit = (int)(floor(u[ax] + 0.5) - c);
    if (bit != 0 && bit != 1) return -1;
    if (copies == 2 && p != 2) {
      // second grid: nearest node of u + 1/2 must be c + 1 (as evaluated by the direct path)
      if (floor((u[ax] + 0.5) + 0.5) != c + 1.0) return -1;
    }
    const int l = (int)c - o[ax];
    if (l < 0 || l >= T) return -1;
    cell = cell * T + l;
    oct = oct * 2 + bit;
  }
  return cell * 8 + oct;
}

// Base node (relative to the cell) and weight polynomials w_s(f) = a0 + a1 f + a2 f^2
// of the order-p kernel on one axis, for grid copy g and octant bit.
__device__ inline int axis_poly(int p, int g, int bit, double (*cf)[3]) {
  if (p == 3) {
    if (g == 0) {
      const double e = 0.5 + bit, h = 0.5 - bit;
      cf[0][0] = 0.5 * e * e; cf[0][1] = -e; cf[0][2] = 0.5;
      cf[1][0] = 0.75 - bit; cf[1][1] = 2.0 * bit; cf[1][2] = -1.0;
      cf[2][0] = 0.5 * h * h; cf[2][1] = h; cf[2][2] = 0.5;
      return bit - 1;
    }
    cf[0][0] = 0.5; cf[0][1] = -1.0; cf[0][2] = 0.5;
    cf[1][0] = 0.5; cf[1][1] = 1.0; cf[1][2] = -1.0;
    cf[2][0] = 0.0; cf[2][1] = 0.0; cf[2][2] = 0.5;
    return 0;
  }
  if (p == 2) {
    if (g == 0) {
      cf[0][0] = 1.0; cf[0][1] = -1.0; cf[0][2] = 0.0;
      cf[1][0] = 0.0; cf[1][1] = 1.0; cf[1][2] = 0.0;
      return 0;
    }
    cf[0][0] = 0.5 + bit; cf[0][1] = -1.0; cf[0][2] = 0.0;
    cf[1][0] = 0.5 - bit; cf[1][1] = 1.0; cf[1][2] = 0.0;
    return bit;
  }
  cf[0][0] = 1.0; cf[0][1] = 0.0; cf[0][2] = 0.0;
  return g == 0 ? bit : 1;
}

// Base node offset (relative to the cell) of axis_poly's stencil.
__device__ inline int axis_base(int p, int g, int bit) {
  if (p == 3) return g == 0 ? bit - 1 : 0;
  if (p == 2) return g == 0 ? 0 : bit;
  return g == 0 ? bit : 1;
}

struct SortArgs {
  const int* start;
  const int* count;
  const double* ux;
  const double* uy;
  const double* uz;
  int T, NT, p, copies, words;
  int* perm;        // records in (cell, octant) order within each tile
  int* ndense;      // [ntiles]
  GroupDesc* desc;  // [ntiles][kMaxDense]
  unsigned* bits;   // [ntiles][words]: key is a moment group
};

// exclusive scan of n ints in LDS by one workgroup (in place), returns the total
__device__ inline int block_scan(int* v, int n, int* tmp) {
  const int t = threadIdx.x;
  const int per = (n + kBlock - 1) / kBlock;
  const int b0 = t * per, b1 = min(n, b0 + per);
  int s = 0;
  for (int i = b0; i < b1; ++i) s += v[i];
  tmp[t] = s;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const int x = t >= off ? tmp[t - off] : 0;
    __syncthreads();
    tmp[t] += x;
    __syncthreads();
  }
  int run = tmp[t] - s;
  const int total = tmp[kBlock - 1];
  __syncthreads();
  for (int i = b0; i < b1; ++i) {
    const int c = v[i];
    v[i] = run;
    run += c;
  }
  __syncthreads();
  return total;
}

__global__ void __launch_bounds__(kBlock) tile_sort_kernel(SortArgs a) {
  extern __shared__ int sh[];
  const int nkeys = 8 * a.T * a.T * a.T;
  int* cnt = sh;                    // [nkeys + 1], last bin: direct path
  int* pos = cnt + nkeys + 1;       // [nkeys + 1]
  int* flag = pos + nkeys + 1;      // [nkeys]
  unsigned* bw = (unsigned*)(flag + nkeys);   // [words]
  __shared__ int tmp[kBlock];
  const int tile = blockIdx.x;
  const int o[3] = {tile / (a.NT * a.NT) * a.T, (tile / a.NT) % a.NT * a.T, tile % a.NT * a.T};
  const int st = a.start[tile], n = a.count[tile];
  for (int i = threadIdx.x; i <= nkeys; i += kBlock) cnt[i] = 0;
  for (int i = threadIdx.x; i < a.words; i += kBlock) bw[i] = 0u;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) {
    const double u[3] = {a.ux[st + i], a.uy[st + i], a.uz[st + i]};
    const int k = group_key(u, o, a.T, a.p, a.copies);
    atomicAdd(&cnt[k < 0 ? nkeys : k], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= nkeys; i += kBlock) {
    pos[i] = cnt[i];
    if (i < nkeys) flag[i] = cnt[i] >= kDenseMin ? 1 : 0;
  }
  __syncthreads();
  block_scan(pos, nkeys + 1, tmp);
  // the first kMaxDense qualifying keys in key order become moment groups
  const int nd = block_scan(flag, nkeys, tmp);
  for (int k = threadIdx.x; k < nkeys; k += kBlock) {
    if (cnt[k] < kDenseMin) continue;
    const int r = flag[k];
    if (r >= kMaxDense) continue;
    GroupDesc d;
    d.start = st + pos[k];
    d.count = cnt[k];
    d.key = k;
    d.pad = 0;
    a.desc[(size_t)tile * kMaxDense + r] = d;
    atomicOr(&bw[k >> 5], 1u << (k & 31));
  }
  __syncthreads();
  if (threadIdx.x == 0) a.ndense[tile] = min(nd, kMaxDense);
  for (int i = threadIdx.x; i < a.words; i += kBlock) a.bits[(size_t)tile * a.words + i] = bw[i];
  // scatter the record indices into key order (order inside a key is immaterial)
  for (int i = threadIdx.x; i <= nkeys; i += kBlock) cnt[i] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) {
    const double u[3] = {a.ux[st + i], a.uy[st + i], a.uz[st + i]};
    int k = group_key(u, o, a.T, a.p, a.copies);
    if (k < 0) k = nkeys;
    const int slot = pos[k] + atomicAdd(&cnt[k], 1);
    a.perm[st + slot] = st + i;
  }
}

template <typename T>
struct MomentArgs {
  const int* dense_off;    // exclusive scan of ndense over tiles
  const int* ndense;
  const GroupDesc* desc;
  const int* perm;
  Records<T> rec;
  int ntiles, tile, NT, p, copies, nchx;   // tile: assignment tile side
  const DevScalars* scal;
  long long* contrib;      // [group][copies][p^3][nchx]
};

// one wavefront (= one workgroup of 64) per moment group
template <typename T>
__global__ void __launch_bounds__(64) dense_moment_kernel(MomentArgs<T> a) {
  __shared__ long long part[64][27];
  __shared__ double mom[27];
  const int lane = threadIdx.x;
  const int total = a.dense_off[a.ntiles - 1] + a.ndense[a.ntiles - 1];
  const int gidx = blockIdx.x;
  if (gidx >= total) return;   // the whole workgroup leaves together
  int lo = 0, hi = a.ntiles;     // dense_off[lo] <= gidx < dense_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a.dense_off[mid] <= gidx) lo = mid;
    else hi = mid;
  }
  const int tile = lo;
  const GroupDesc d = a.desc[(size_t)tile * kMaxDense + (gidx - a.dense_off[tile])];
  const int cellk = d.key >> 3, oct = d.key & 7;
  const int ts = a.tile;
  const double c[3] = {(double)(tile / (a.NT * a.NT) * ts + cellk / (ts * ts)),
                       (double)((tile / a.NT) % a.NT * ts + (cellk / ts) % ts),
                       (double)(tile % a.NT * ts + cellk % ts)};
  const int bits[3] = {(oct >> 2) & 1, (oct >> 1) & 1, oct & 1};
  const double scale = a.scal->scale, inv_scale = a.scal->inv_scale;
  const int np = a.p * a.p * a.p;
  for (int ch = 0; ch < a.nchx; ++ch) {
    long long m[27];
#pragma unroll
    for (int j = 0; j < 27; ++j) m[j] = 0;
    for (int i = lane; i < d.count; i += 64) {
      const int r = a.perm[d.start + i];
      const double cv = (double)a.rec.cv[(int64_t)ch * a.rec.cap + r];
      const double f[3] = {a.rec.ux[r] - c[0], a.rec.uy[r] - c[1], a.rec.uz[r] - c[2]};
      const double px[3] = {1.0, f[0], f[0] * f[0]}, py[3] = {1.0, f[1], f[1] * f[1]},
                   pz[3] = {1.0, f[2], f[2] * f[2]};
#pragma unroll
      for (int ia = 0; ia < 3; ++ia)
#pragma unroll
        for (int ib = 0; ib < 3; ++ib)
#pragma unroll
          for (int ic = 0; ic < 3; ++ic) m[(ia * 3 + ib) * 3 + ic] += llrint(cv * px[ia] * py[ib] * pz[ic] * scale);
    }
#pragma unroll
    for (int j = 0; j < 27; ++j) part[lane][j] = m[j];
    __syncthreads();
    if (lane < 27) {
      long long sum = 0;
      for (int l = 0; l < 64; ++l) sum += part[l][lane];
      mom[lane] = (double)sum * inv_scale;
    }
    __syncthreads();
    // node contributions of both grid copies
    for (int item = lane; item < a.copies * np; item += 64) {
      const int g = item / np, nd = item % np;
      const int sx = nd / (a.p * a.p), sy = (nd / a.p) % a.p, sz = nd % a.p;
      double cx[3][3], cy[3][3], cz[3][3];
      axis_poly(a.p, g, bits[0], cx);
      axis_poly(a.p, g, bits[1], cy);
      axis_poly(a.p, g, bits[2], cz);
      double v = 0.0;
      for (int ia = 0; ia < 3; ++ia)
        for (int ib = 0; ib < 3; ++ib)
          for (int ic = 0; ic < 3; ++ic) v += cx[sx][ia] * cy[sy][ib] * cz[sz][ic] * mom[(ia * 3 + ib) * 3 + ic];
      a.contrib[(((size_t)gidx * a.copies + g) * np + nd) * a.nchx + ch] = llrint(v * scale);
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// tile assignment

struct TileArgs {
  double inv_h, h, origin[3];
  int N, T, NT, p, copies, box_mode;
  ChanInfo ci;
  int ngrid;
  int gre[kMaxGrids], gim[kMaxGrids];
  const int* start;
  const int* count;
  const DevScalars* scal;
  void* out;                   // [copies][ngrid][N^3] complex
  double* tile_I;              // survey: per-tile sum of (alpha R)^3
  // moment groups
  const int* ndense;
  const int* dense_off;
  const GroupDesc* desc;
  const unsigned* bits;
  int words;
  const long long* contrib;
};

// Per-axis stencil of the order-p kernel (Hockney & Eastwood) at grid
// coordinate u: lowest node index j0 (unwrapped) and weights.
__device__ inline int axis_stencil(double u, int p, double* wt) {
  if (p == 1) {
    wt[0] = 1.0;
    return (int)floor(u + 0.5);
  }
  if (p == 2) {
    const double j = floor(u), d = u - j;
    wt[0] = 1.0 - d;
    wt[1] = d;
    return (int)j;
  }
  const double j = floor(u + 0.5), d = u - j;
  wt[0] = 0.5 * (0.5 - d) * (0.5 - d);
  wt[1] = 0.75 - d * d;
  wt[2] = 0.5 * (0.5 + d) * (0.5 + d);
  return (int)j - 1;
}

// Box mode (periodic, no randoms): dn = n - nbar subtracts the mean weight per
// cell times y_L^M*(x^_node) from channel ch.
__device__ inline double node_term(const ChanInfo& ci, int ch, double mean, double ux, double uy, double uz) {
  double re = 1.0, im = 0.0;
  if (ci.local) ylm_pos_m(ci.chL[ch], ci.chM[ch], ux, uy, uz, ci.ynorm, &re, &im);
  return mean * (ci.chPart[ch] ? -im : re);
}

template <typename T, int NCH>
__global__ void __launch_bounds__(kBlock) assign_tile_kernel(TileArgs a, Records<T> rec) {
  typedef typename cplx<T>::type T2;
  extern __shared__ unsigned long long acc[];   // [copies][nchx][T^3]
  __shared__ int nb_start[27];
  __shared__ int nb_off[28];
  __shared__ int nb_tile[27];
  __shared__ int nb_org[27][3];
  __shared__ int nb_goff[28];                   // prefix of the neighbours' moment-group items
  const int T3 = a.T * a.T * a.T;
  const int nch = a.ci.nch;
  const int nchx = nch + (a.box_mode ? 0 : 1);
  const int tile = blockIdx.x;
  const int tx = tile / (a.NT * a.NT), ty = (tile / a.NT) % a.NT, tz = tile % a.NT;
  const int ox = tx * a.T, oy = ty * a.T, oz = tz * a.T;
  const int N = a.N;
  for (int i = threadIdx.x; i < a.copies * nchx * T3; i += kBlock) acc[i] = 0ull;
  // the 27 neighbouring tiles, each once even when NT < 3 wraps them together
  if (threadIdx.x < 27) {
    const int nb = threadIdx.x;
    const int nx = (tx + nb / 9 - 1 + a.NT) % a.NT, ny = (ty + (nb / 3) % 3 - 1 + a.NT) % a.NT,
              nz = (tz + nb % 3 - 1 + a.NT) % a.NT;
    bool dup = false;
    for (int pb = 0; pb < nb && !dup; ++pb) {
      const int ex = (tx + pb / 9 - 1 + a.NT) % a.NT, ey = (ty + (pb / 3) % 3 - 1 + a.NT) % a.NT,
                ez = (tz + pb % 3 - 1 + a.NT) % a.NT;
      dup = (ex == nx && ey == ny && ez == nz);
    }
    const int nt = (nx * a.NT + ny) * a.NT + nz;
    nb_start[nb] = a.start[nt];
    nb_off[nb + 1] = dup ? 0 : a.count[nt];
    nb_tile[nb] = nt;
    nb_org[nb][0] = nx * a.T;
    nb_org[nb][1] = ny * a.T;
    nb_org[nb][2] = nz * a.T;
    nb_goff[nb + 1] = dup ? 0 : a.ndense[nt];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    nb_off[0] = 0;
    nb_goff[0] = 0;
    for (int k = 0; k < 27; ++k) {
      nb_off[k + 1] += nb_off[k];
      nb_goff[k + 1] += nb_goff[k];
    }
  }
  __syncthreads();
  const double scale = a.scal->scale;
  const int total = nb_off[27];
  for (int idx = threadIdx.x; idx < total; idx += kBlock) {
    int lo = 0, hi = 27;   // nb_off[lo] <= idx < nb_off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (nb_off[mid] <= idx) lo = mid;
      else hi = mid;
    }
    const int64_t slot = nb_start[lo] + (idx - nb_off[lo]);
    const double u[3] = {rec.ux[slot], rec.uy[slot], rec.uz[slot]};
    if (!isfinite(u[0])) continue;
    {
      // particles of their tile's moment groups arrive through the group sums below
      const int key = group_key(u, nb_org[lo], a.T, a.p, a.copies);
      if (key >= 0 && (a.bits[(size_t)nb_tile[lo] * a.words + (key >> 5)] >> (key & 31) & 1u)) continue;
    }
    bool have = false;
    double cv[NCH];
    for (int g = 0; g < a.copies; ++g) {
      double wt[3][3];
      int lo3[3], msk[3];
      bool any = true;
      const int o3[3] = {ox, oy, oz};
      for (int ax = 0; ax < 3; ++ax) {
        lo3[ax] = axis_stencil(u[ax] + 0.5 * g, a.p, wt[ax]);
        msk[ax] = 0;
        for (int s = 0; s < a.p; ++s) {
          int jj = lo3[ax] + s;
          if (jj < 0) jj += N;
          if (jj >= N) jj -= N;
          const int l = jj - o3[ax];
          if (l >= 0 && l < a.T) msk[ax] |= 1 << s;
        }
        any = any && msk[ax];
      }
      if (!any) continue;
      if (!have) {
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) cv[ch] = ch < nchx ? (double)rec.cv[(int64_t)ch * rec.cap + slot] : 0.0;
        have = true;
      }
      for (int sx = 0; sx < a.p; ++sx) {
        if (!(msk[0] >> sx & 1)) continue;
        int jx = lo3[0] + sx;
        jx += jx < 0 ? N : (jx >= N ? -N : 0);
        const int lx = jx - ox;
        for (int sy = 0; sy < a.p; ++sy) {
          if (!(msk[1] >> sy & 1)) continue;
          int jy = lo3[1] + sy;
          jy += jy < 0 ? N : (jy >= N ? -N : 0);
          const int ly = jy - oy;
          const double wxy = wt[0][sx] * wt[1][sy];
          for (int sz = 0; sz < a.p; ++sz) {
            if (!(msk[2] >> sz & 1)) continue;
            int jz = lo3[2] + sz;
            jz += jz < 0 ? N : (jz >= N ? -N : 0);
            const int lz = jz - oz;
            const double W = wxy * wt[2][sz];
            const int cell = (lx * a.T + ly) * a.T + lz;
            unsigned long long* base = acc + (size_t)g * nchx * T3 + cell;
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
              if (ch >= nchx) break;
              if (ch == nch && g != 0) break;
              const double v = cv[ch] * W;
              if (v != 0.0) atomicAdd(base + (size_t)ch * T3, (unsigned long long)llrint(v * scale));
            }
          }
        }
      }
    }
  }
  // moment groups of the neighbouring tiles: add their node sums that fall here
  {
    const int np = a.p * a.p * a.p;
    const int per_group = a.copies * np;
    const int gtotal = nb_goff[27] * per_group;
    for (int item = threadIdx.x; item < gtotal; item += kBlock) {
      const int gi = item / per_group, rest = item - gi * per_group;
      const int g = rest / np, nd = rest - g * np;
      int lo = 0, hi = 27;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (nb_goff[mid] <= gi) lo = mid;
        else hi = mid;
      }
      const int nt = nb_tile[lo];
      const int j = gi - nb_goff[lo];
      const GroupDesc d = a.desc[(size_t)nt * kMaxDense + j];
      const int cellk = d.key >> 3, oct = d.key & 7;
      const int sv[3] = {nd / (a.p * a.p), (nd / a.p) % a.p, nd % a.p};
      const int loc[3] = {cellk / (a.T * a.T), (cellk / a.T) % a.T, cellk % a.T};
      const int o3[3] = {ox, oy, oz};
      int l3[3];
      bool inside = true;
      for (int ax = 0; ax < 3; ++ax) {
        const int bit = (oct >> (2 - ax)) & 1;
        int jj = nb_org[lo][ax] + loc[ax] + axis_base(a.p, g, bit) + sv[ax];
        jj += jj < 0 ? N : (jj >= N ? -N : 0);
        l3[ax] = jj - o3[ax];
        inside = inside && l3[ax] >= 0 && l3[ax] < a.T;
      }
      if (!inside) continue;
      const int cell = (l3[0] * a.T + l3[1]) * a.T + l3[2];
      const long long* cb = a.contrib + (((size_t)(a.dense_off[nt] + j) * a.copies + g) * np + nd) * nchx;
      unsigned long long* base = acc + (size_t)g * nchx * T3 + cell;
      for (int ch = 0; ch < nchx; ++ch) {
        if (ch == nch && g != 0) break;
        const long long v = cb[ch];
        if (v != 0) atomicAdd(base + (size_t)ch * T3, (unsigned long long)v);
      }
    }
  }
  __syncthreads();

  // write out: value = sum / scale - (box mode) (sum w / N^3) y_L^M*(x^_node)
  const double inv_scale = a.scal->inv_scale;
  const double mean = a.scal->mean_cell;
  T2* out = (T2*)a.out;
  const size_t N3 = (size_t)N * N * N;
  for (int i = threadIdx.x; i < a.copies * T3; i += kBlock) {
    const int g = i / T3, cell = i % T3;
    const int lx = cell / (a.T * a.T), ly = (cell / a.T) % a.T, lz = cell % a.T;
    const int ix = ox + lx, iy = oy + ly, iz = oz + lz;
    double ux = 0.0, uy = 0.0, uz = 1.0;
    if (a.box_mode && a.ci.local) {
      const double px = a.origin[0] + (ix - 0.5 * g) * a.h - a.ci.obs[0];
      const double py = a.origin[1] + (iy - 0.5 * g) * a.h - a.ci.obs[1];
      const double pz = a.origin[2] + (iz - 0.5 * g) * a.h - a.ci.obs[2];
      const double r = sqrt(px * px + py * py + pz * pz);
      if (r > 0.0) {
        ux = px / r;
        uy = py / r;
        uz = pz / r;
      }
    }
    const size_t lin = ((size_t)ix * N + iy) * N + iz;
    for (int gr = 0; gr < a.ngrid; ++gr) {
      const int cre = a.gre[gr], cim = a.gim[gr];
      double vre = (double)(long long)acc[((size_t)g * nchx + cre) * T3 + cell] * inv_scale;
      double vim = cim >= 0 ? (double)(long long)acc[((size_t)g * nchx + cim) * T3 + cell] * inv_scale : 0.0;
      if (a.box_mode) {
        vre -= node_term(a.ci, cre, mean, ux, uy, uz);
        if (cim >= 0) vim -= node_term(a.ci, cim, mean, ux, uy, uz);
      }
      T2 o;
      o.x = (T)vre;
      o.y = (T)vim;
      out[((size_t)g * a.ngrid + gr) * N3 + lin] = o;
    }
  }
  if (!a.box_mode) {
    // Sec. 4.2, eq. 37: partial of sum_j (alpha R_j)^3 over this tile (first grid)
    __shared__ double sh[kBlock];
    const double alpha = a.scal->alpha;
    double s = 0.0;
    for (int cell = threadIdx.x; cell < T3; cell += kBlock) {
      const double R = (double)(long long)acc[(size_t)nch * T3 + cell] * inv_scale;
      const double v = alpha * R;
      s += v * v * v;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
      if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.tile_I[tile] = sh[0];
  }
}

__global__ void __launch_bounds__(kBlock) norm_final_kernel(const double* tile_I, int ntiles,
                                                            DevScalars* scal, double vc) {
  __shared__ double sh[kBlock];
  double s = 0.0;
  for (int t = threadIdx.x; t < ntiles; t += kBlock) s += tile_I[t];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) scal->I = sh[0] / (vc * vc);   // I = v_c sum (alpha R / v_c)^3
}

__global__ void zero_ints_kernel(int* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void zero_scal_kernel(DevScalars* s) {
  if (threadIdx.x == 0) {
    s->sum_w = s->sum_w_ran = s->sum_abs = s->sum_abs_ran = 0.0;
    s->alpha = s->scale = s->inv_scale = s->mean_cell = s->I = 0.0;
    s->err = 0;
    s->pad = 0;
  }
}

struct GridMap {
  int gre[kMaxGrids], gim[kMaxGrids];
};

template <typename T>
__global__ void unpack_kernel(const void* grid, void* out, int copies, int ngrid, GridMap m,
                              int nch, int64_t N3) {
  typedef typename cplx<T>::type T2;
  const T2* g = (const T2*)grid;
  T* o = (T*)out;
  const int64_t total = (int64_t)copies * ngrid * N3;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cell = i % N3;
    const int64_t cg = i / N3;
    const int c = (int)(cg / ngrid), gr = (int)(cg % ngrid);
    const T2 v = g[i];
    o[((int64_t)c * nch + m.gre[gr]) * N3 + cell] = v.x;
    if (m.gim[gr] >= 0) o[((int64_t)c * nch + m.gim[gr]) * N3 + cell] = v.y;
  }
}

int grid_blocks(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b > 4096) b = 4096;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

int run_prep(Plan& P, const tsb_catalog* data, const tsb_catalog* rand, hipStream_t s) {
  PrepArgs a{};
  a.d = cat_ptrs(data);
  a.r = P.box_mode ? CatPtrs{} : cat_ptrs(rand);
  a.P0 = P.P0;
  a.inv_h = (double)P.N / P.L;
  for (int i = 0; i < 3; ++i) {
    a.origin[i] = P.origin[i];
    a.obs[i] = P.observer[i];
  }
  a.N = P.N;
  a.box_mode = P.box_mode;
  a.local = P.los_kind == TSB_LOS_LOCAL;
  a.scal = P.d_scal;
  a.partials = P.d_sum_partials;
  prof_begin(P, kStWeights, s);
  hipLaunchKernelGGL(zero_scal_kernel, dim3(1), dim3(64), 0, s, P.d_scal);
  hipLaunchKernelGGL(prep_kernel, dim3(kPrepBlocks), dim3(kBlock), 0, s, a);
  const double n3 = (double)P.N * P.N * P.N;
  hipLaunchKernelGGL(prep_final_kernel, dim3(1), dim3(kBlock), 0, s, (const double*)P.d_sum_partials,
                     kPrepBlocks, P.d_scal, P.box_mode, n3, P.L * P.L * P.L);
  prof_end(P, kStWeights, s);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

template <typename T, int NCH>
int assign_impl(Plan& P, const BucketArgs& b, const ChanInfo& ci, hipStream_t s) {
  const int ntiles = P.NT * P.NT * P.NT;
  const int64_t ntot = b.d.n + b.r.n;
  const int nchx = ci.nch + (P.box_mode ? 0 : 1);
  Records<T> rec;
  rec.cap = P.particle_cap;
  rec.ux = (double*)P.d_rec_u;
  rec.uy = rec.ux + rec.cap;
  rec.uz = rec.uy + rec.cap;
  rec.cv = (T*)P.d_rec_c;
  if (ntot > 0) {
    FillArgs<T, NCH> f;
    f.b = b;
    f.ci = ci;
    f.rec = rec;
    f.P0 = P.P0;
    f.box_mode = P.box_mode;
    f.nchx = nchx;
    f.scal = P.d_scal;
    hipLaunchKernelGGL((bucket_fill_kernel<T, NCH>), dim3(grid_blocks(ntot)), dim3(kBlock), 0, s, f);
  }
  // moment groups: per-tile sort by (cell, octant), then one wavefront per group
  const int words = 8 * P.T * P.T * P.T / 32;
  {
    SortArgs so;
    so.start = P.d_tile_start;
    so.count = P.d_tile_count;
    so.ux = rec.ux;
    so.uy = rec.uy;
    so.uz = rec.uz;
    so.T = P.T;
    so.NT = P.NT;
    so.p = P.p;
    so.copies = P.copies;
    so.words = words;
    so.perm = P.d_perm;
    so.ndense = P.d_tile_ndense;
    so.desc = (GroupDesc*)P.d_dense_desc;
    so.bits = (unsigned*)P.d_dense_bits;
    const int nkeys = 8 * P.T * P.T * P.T;
    const size_t lds = (size_t)(3 * nkeys + 2) * sizeof(int) + (size_t)words * sizeof(unsigned);
    hipLaunchKernelGGL(tile_sort_kernel, dim3(ntiles), dim3(kBlock), lds, s, so);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, (const int*)P.d_tile_ndense, P.d_dense_off, ntiles);
    MomentArgs<T> m;
    m.dense_off = P.d_dense_off;
    m.ndense = P.d_tile_ndense;
    m.desc = (const GroupDesc*)P.d_dense_desc;
    m.perm = P.d_perm;
    m.rec = rec;
    m.ntiles = ntiles;
    m.tile = P.T;
    m.NT = P.NT;
    m.p = P.p;
    m.copies = P.copies;
    m.nchx = nchx;
    m.scal = P.d_scal;
    m.contrib = (long long*)P.d_dense_contrib;
    const int64_t groups = std::min<int64_t>((int64_t)ntiles * kMaxDense, ntot / kDenseMin + 1);
    hipLaunchKernelGGL(dense_moment_kernel<T>, dim3((unsigned)groups), dim3(64), 0, s, m);
  }
  prof_end(P, kStBucket, s);

  TileArgs a{};
  a.inv_h = (double)P.N / P.L;
  a.h = P.L / (double)P.N;
  for (int i = 0; i < 3; ++i) a.origin[i] = P.origin[i];
  a.N = P.N;
  a.T = P.T;
  a.NT = P.NT;
  a.p = P.p;
  a.copies = P.copies;
  a.box_mode = P.box_mode;
  a.ci = ci;
  a.ngrid = (int)P.grids.size();
  for (int g = 0; g < a.ngrid; ++g) {
    a.gre[g] = P.grids[g].re;
    a.gim[g] = P.grids[g].im;
  }
  a.start = P.d_tile_start;
  a.count = P.d_tile_count;
  a.scal = P.d_scal;
  a.out = P.d_grid;
  a.tile_I = P.d_sum_partials;
  a.ndense = P.d_tile_ndense;
  a.dense_off = P.d_dense_off;
  a.desc = (const GroupDesc*)P.d_dense_desc;
  a.bits = (const unsigned*)P.d_dense_bits;
  a.words = words;
  a.contrib = (const long long*)P.d_dense_contrib;
  const size_t lds = (size_t)P.copies * nchx * P.T * P.T * P.T * sizeof(unsigned long long);
  prof_begin(P, kStAssign, s);
  hipLaunchKernelGGL((assign_tile_kernel<T, NCH>), dim3(ntiles), dim3(kBlock), lds, s, a, rec);
  if (!P.box_mode) {
    const double vc = P.L * P.L * P.L / ((double)P.N * P.N * P.N);
    hipLaunchKernelGGL(norm_final_kernel, dim3(1), dim3(kBlock), 0, s, (const double*)P.d_sum_partials,
                       ntiles, P.d_scal, vc);
  }
  prof_end(P, kStAssign, s);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

int run_assign(Plan& P, const tsb_catalog* data, const tsb_catalog* rand, hipStream_t s) {
  const int ntiles = P.NT * P.NT * P.NT;
  BucketArgs b{};
  b.d = cat_ptrs(data);
  b.r = P.box_mode ? CatPtrs{} : cat_ptrs(rand);
  b.inv_h = (double)P.N / P.L;
  for (int i = 0; i < 3; ++i) b.origin[i] = P.origin[i];
  b.N = P.N;
  b.T = P.T;
  b.NT = P.NT;
  b.count = P.d_tile_count;
  b.cursor = P.d_tile_cursor;
  b.start = P.d_tile_start;
  b.keys = P.d_keys;
  const int64_t ntot = b.d.n + b.r.n;
  prof_begin(P, kStBucket, s);
  hipLaunchKernelGGL(zero_ints_kernel, dim3(grid_blocks(ntiles)), dim3(kBlock), 0, s, P.d_tile_count, (int64_t)ntiles);
  hipLaunchKernelGGL(zero_ints_kernel, dim3(grid_blocks(ntiles)), dim3(kBlock), 0, s, P.d_tile_cursor, (int64_t)ntiles);
  if (ntot > 0)
    hipLaunchKernelGGL(bucket_count_kernel, dim3(grid_blocks(ntot)), dim3(kBlock), 0, s, b);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, (const int*)P.d_tile_count, P.d_tile_start, ntiles);

  ChanInfo ci{};
  ci.nch = (int)P.chans.size();
  if (ci.nch + 1 > kMaxCh || (int)P.grids.size() > kMaxGrids) return fail(TSB_E_UNSUPPORTED, "too many channels");
  ci.local = P.los_kind == TSB_LOS_LOCAL;
  for (int i = 0; i < 3; ++i) ci.obs[i] = P.observer[i];
  for (int c = 0; c < ci.nch; ++c) {
    ci.chL[c] = P.chans[c].L;
    ci.chM[c] = P.chans[c].M;
    ci.chPart[c] = P.chans[c].part;
  }
  ylm_norm_table(ci.ynorm);
  const int nchx = ci.nch + (P.box_mode ? 0 : 1);
  const bool f64 = P.precision == TSB_FP64;
  if (nchx <= 8) return f64 ? assign_impl<double, 8>(P, b, ci, s) : assign_impl<float, 8>(P, b, ci, s);
  if (nchx <= 16) return f64 ? assign_impl<double, 16>(P, b, ci, s) : assign_impl<float, 16>(P, b, ci, s);
  return f64 ? assign_impl<double, kMaxCh>(P, b, ci, s) : assign_impl<float, kMaxCh>(P, b, ci, s);
}

int run_unpack_grids(Plan& P, void* out, hipStream_t s) {
  const int64_t N3 = (int64_t)P.N * P.N * P.N;
  GridMap m{};
  for (size_t g = 0; g < P.grids.size(); ++g) {
    m.gre[g] = P.grids[g].re;
    m.gim[g] = P.grids[g].im;
  }
  const int64_t total = (int64_t)P.copies * (int64_t)P.grids.size() * N3;
  if (P.precision == TSB_FP64)
    hipLaunchKernelGGL(unpack_kernel<double>, dim3(grid_blocks(total)), dim3(kBlock), 0, s,
                       (const void*)P.d_grid, out, P.copies, (int)P.grids.size(), m, (int)P.chans.size(), N3);
  else
    hipLaunchKernelGGL(unpack_kernel<float>, dim3(grid_blocks(total)), dim3(kBlock), 0, s,
                       (const void*)P.d_grid, out, P.copies, (int)P.grids.size(), m, (int)P.chans.size(), N3);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

}  // namespace tsb
