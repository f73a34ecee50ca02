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
  int* sorted;
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

__global__ void __launch_bounds__(kBlock) bucket_fill_kernel(BucketArgs a) {
  const int64_t ntot = a.d.n + a.r.n;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < ntot;
       i += (int64_t)gridDim.x * kBlock) {
    const int key = a.keys[i];
    const int slot = a.start[key] + atomicAdd(&a.cursor[key], 1);
    a.sorted[slot] = (int)i;
  }
}

// ----------------------------------------------------------------------------
// tile assignment

struct TileArgs {
  CatPtrs d, r;
  double P0, inv_h, h, origin[3], obs[3];
  int N, T, NT, p, copies, box_mode, local;
  int nch;                     // real channels (the survey randoms channel is nch)
  int chL[kMaxCh], chM[kMaxCh], chPart[kMaxCh];
  int ngrid;
  int gre[kMaxGrids], gim[kMaxGrids];
  double ynorm[45];
  const int* start;
  const int* count;
  const int* sorted;
  const DevScalars* scal;
  void* out;                   // [copies][ngrid][N^3] complex
  double* tile_I;              // survey: per-tile sum of (alpha R)^3
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

template <int NCH>
__device__ inline void channel_values(const TileArgs& a, double x, double y, double z, double w,
                                      bool ran, double alpha, double* cv) {
  // c = w y_L^M*(x^) (eq. 34); randoms carry -alpha (eq. 34), plus the
  // unweighted-by-y randoms channel for the normalisation (survey mode)
  double ux = 0.0, uy = 0.0, uz = 1.0;
  if (a.local) {
    const double dx = x - a.obs[0], dy = y - a.obs[1], dz = z - a.obs[2];
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
    if (c >= a.nch) {
      cv[c] = (c == a.nch && ran) ? w : 0.0;
      continue;
    }
    double re = 1.0, im = 0.0;
    if (a.local) ylm_pos_m(a.chL[c], a.chM[c], ux, uy, uz, a.ynorm, &re, &im);
    // Re(y*) = Re(y), Im(y*) = -Im(y)
    cv[c] = s * (a.chPart[c] ? -im : re);
  }
}

// Box mode (periodic, no randoms): dn = n - nbar subtracts the mean weight per
// cell times y_L^M*(x^_node) from channel ch.
__device__ inline double node_term(const TileArgs& a, int ch, double mean, double ux, double uy,
                                   double uz) {
  double re = 1.0, im = 0.0;
  if (a.local) ylm_pos_m(a.chL[ch], a.chM[ch], ux, uy, uz, a.ynorm, &re, &im);
  return mean * (a.chPart[ch] ? -im : re);
}

template <typename T, int NCH>
__global__ void __launch_bounds__(kBlock) assign_tile_kernel(TileArgs a) {
  typedef typename cplx<T>::type T2;
  extern __shared__ unsigned long long acc[];   // [copies][nchx][T^3]
  const int T3 = a.T * a.T * a.T;
  const int nchx = a.nch + (a.box_mode ? 0 : 1);
  const int tile = blockIdx.x;
  const int tx = tile / (a.NT * a.NT), ty = (tile / a.NT) % a.NT, tz = tile % a.NT;
  const int ox = tx * a.T, oy = ty * a.T, oz = tz * a.T;
  for (int i = threadIdx.x; i < a.copies * nchx * T3; i += kBlock) acc[i] = 0ull;
  __syncthreads();
  const double scale = a.scal->scale;
  const double alpha = a.scal->alpha;

  // neighbouring tiles, each visited once even when NT < 3 wraps them together
  for (int nb = 0; nb < 27; ++nb) {
    const int dx = nb / 9 - 1, dy = (nb / 3) % 3 - 1, dz = nb % 3 - 1;
    const int nx = (tx + dx + a.NT) % a.NT, ny = (ty + dy + a.NT) % a.NT, nz = (tz + dz + a.NT) % a.NT;
    bool dup = false;
    for (int pb = 0; pb < nb && !dup; ++pb) {
      const int ex = (tx + pb / 9 - 1 + a.NT) % a.NT, ey = (ty + (pb / 3) % 3 - 1 + a.NT) % a.NT,
                ez = (tz + pb % 3 - 1 + a.NT) % a.NT;
      dup = (ex == nx && ey == ny && ez == nz);
    }
    if (dup) continue;
    const int nt = (nx * a.NT + ny) * a.NT + nz;
    const int st = a.start[nt], cnt = a.count[nt];
    for (int k = threadIdx.x; k < cnt; k += kBlock) {
      const int pid = a.sorted[st + k];
      const bool ran = pid >= a.d.n;
      const CatPtrs& c = ran ? a.r : a.d;
      const int64_t j = ran ? (int64_t)pid - a.d.n : (int64_t)pid;
      const double x = c.x[j], y = c.y[j], z = c.z[j];
      const double w = particle_weight(c, j, a.P0);
      double u[3] = {(x - a.origin[0]) * a.inv_h, (y - a.origin[1]) * a.inv_h,
                     (z - a.origin[2]) * a.inv_h};
      bool ok = isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]) && isfinite(w);
      for (int ax = 0; ax < 3 && ok; ++ax) {
        if (u[ax] < 0.0 || u[ax] >= a.N) {
          if (!a.box_mode) ok = false;   // reported by the weight pass
          else u[ax] -= a.N * floor(u[ax] / a.N);
        }
      }
      if (!ok) continue;
      double cv[NCH];
      bool have = false;
      for (int g = 0; g < a.copies; ++g) {
        double wt[3][3];
        int lo[3], msk[3];
        bool any = true;
        for (int ax = 0; ax < 3; ++ax) {
          const double ug = u[ax] + 0.5 * g;
          lo[ax] = axis_stencil(ug, a.p, wt[ax]);
          const int o = ax == 0 ? ox : (ax == 1 ? oy : oz);
          msk[ax] = 0;
          for (int s = 0; s < a.p; ++s) {
            int jj = (lo[ax] + s) % a.N;
            if (jj < 0) jj += a.N;
            const int l = jj - o;
            if (l >= 0 && l < a.T) msk[ax] |= 1 << s;
          }
          any = any && msk[ax];
        }
        if (!any) continue;
        if (!have) {
          channel_values<NCH>(a, x, y, z, w, ran, alpha, cv);
          have = true;
        }
        for (int sx = 0; sx < a.p; ++sx) {
          if (!(msk[0] >> sx & 1)) continue;
          const int lx = ((lo[0] + sx) % a.N + a.N) % a.N - ox;
          for (int sy = 0; sy < a.p; ++sy) {
            if (!(msk[1] >> sy & 1)) continue;
            const int ly = ((lo[1] + sy) % a.N + a.N) % a.N - oy;
            const double wxy = wt[0][sx] * wt[1][sy];
            for (int sz = 0; sz < a.p; ++sz) {
              if (!(msk[2] >> sz & 1)) continue;
              const int lz = ((lo[2] + sz) % a.N + a.N) % a.N - oz;
              const double W = wxy * wt[2][sz];
              const int cell = (lx * a.T + ly) * a.T + lz;
              unsigned long long* base = acc + (size_t)g * nchx * T3 + cell;
#pragma unroll
              for (int ch = 0; ch < NCH; ++ch) {
                if (ch >= nchx) break;
                if (ch == a.nch && g != 0) break;
                const double v = cv[ch] * W;
                if (v != 0.0)
                  atomicAdd(base + (size_t)ch * T3, (unsigned long long)llrint(v * scale));
              }
            }
          }
        }
      }
    }
  }
  __syncthreads();

  // write out: value = sum / scale - (box mode) (sum w / N^3) y_L^M*(x^_node)
  const double inv_scale = a.scal->inv_scale;
  const double mean = a.scal->mean_cell;
  T2* out = (T2*)a.out;
  const size_t N3 = (size_t)a.N * a.N * a.N;
  for (int i = threadIdx.x; i < a.copies * T3; i += kBlock) {
    const int g = i / T3, cell = i % T3;
    const int lx = cell / (a.T * a.T), ly = (cell / a.T) % a.T, lz = cell % a.T;
    const int ix = ox + lx, iy = oy + ly, iz = oz + lz;
    double ux = 0.0, uy = 0.0, uz = 1.0;
    if (a.box_mode && a.local) {
      const double px = a.origin[0] + (ix - 0.5 * g) * a.h - a.obs[0];
      const double py = a.origin[1] + (iy - 0.5 * g) * a.h - a.obs[1];
      const double pz = a.origin[2] + (iz - 0.5 * g) * a.h - a.obs[2];
      const double r = sqrt(px * px + py * py + pz * pz);
      if (r > 0.0) {
        ux = px / r;
        uy = py / r;
        uz = pz / r;
      }
    }
    const size_t lin = ((size_t)ix * a.N + iy) * a.N + iz;
    for (int gr = 0; gr < a.ngrid; ++gr) {
      const int cre = a.gre[gr], cim = a.gim[gr];
      double vre = (double)(long long)acc[((size_t)g * nchx + cre) * T3 + cell] * inv_scale;
      double vim = cim >= 0 ? (double)(long long)acc[((size_t)g * nchx + cim) * T3 + cell] * inv_scale : 0.0;
      if (a.box_mode) {
        vre -= node_term(a, cre, mean, ux, uy, uz);
        if (cim >= 0) vim -= node_term(a, cim, mean, ux, uy, uz);
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
    double s = 0.0;
    for (int cell = threadIdx.x; cell < T3; cell += kBlock) {
      const double R = (double)(long long)acc[(size_t)a.nch * T3 + cell] * inv_scale;
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
  b.sorted = P.d_sorted;
  const int64_t ntot = b.d.n + b.r.n;
  prof_begin(P, kStBucket, s);
  hipLaunchKernelGGL(zero_ints_kernel, dim3(grid_blocks(ntiles)), dim3(kBlock), 0, s, P.d_tile_count, (int64_t)ntiles);
  hipLaunchKernelGGL(zero_ints_kernel, dim3(grid_blocks(ntiles)), dim3(kBlock), 0, s, P.d_tile_cursor, (int64_t)ntiles);
  if (ntot > 0)
    hipLaunchKernelGGL(bucket_count_kernel, dim3(grid_blocks(ntot)), dim3(kBlock), 0, s, b);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, (const int*)P.d_tile_count, P.d_tile_start, ntiles);
  if (ntot > 0)
    hipLaunchKernelGGL(bucket_fill_kernel, dim3(grid_blocks(ntot)), dim3(kBlock), 0, s, b);
  prof_end(P, kStBucket, s);

  TileArgs a{};
  a.d = b.d;
  a.r = b.r;
  a.P0 = P.P0;
  a.inv_h = (double)P.N / P.L;
  a.h = P.L / (double)P.N;
  for (int i = 0; i < 3; ++i) {
    a.origin[i] = P.origin[i];
    a.obs[i] = P.observer[i];
  }
  a.N = P.N;
  a.T = P.T;
  a.NT = P.NT;
  a.p = P.p;
  a.copies = P.copies;
  a.box_mode = P.box_mode;
  a.local = P.los_kind == TSB_LOS_LOCAL;
  a.nch = (int)P.chans.size();
  if (a.nch + 1 > kMaxCh || (int)P.grids.size() > kMaxGrids)
    return fail(TSB_E_UNSUPPORTED, "too many channels");
  for (int c = 0; c < a.nch; ++c) {
    a.chL[c] = P.chans[c].L;
    a.chM[c] = P.chans[c].M;
    a.chPart[c] = P.chans[c].part;
  }
  a.ngrid = (int)P.grids.size();
  for (int g = 0; g < a.ngrid; ++g) {
    a.gre[g] = P.grids[g].re;
    a.gim[g] = P.grids[g].im;
  }
  ylm_norm_table(a.ynorm);
  a.start = P.d_tile_start;
  a.count = P.d_tile_count;
  a.sorted = P.d_sorted;
  a.scal = P.d_scal;
  a.out = P.d_grid;
  a.tile_I = P.d_sum_partials;
  const int nchx = a.nch + (P.box_mode ? 0 : 1);
  const size_t lds = (size_t)P.copies * nchx * P.T * P.T * P.T * sizeof(unsigned long long);
  const bool f64 = P.precision == TSB_FP64;
  prof_begin(P, kStAssign, s);
  if (nchx <= 8) {
    if (f64) hipLaunchKernelGGL((assign_tile_kernel<double, 8>), dim3(ntiles), dim3(kBlock), lds, s, a);
    else hipLaunchKernelGGL((assign_tile_kernel<float, 8>), dim3(ntiles), dim3(kBlock), lds, s, a);
  } else if (nchx <= 16) {
    if (f64) hipLaunchKernelGGL((assign_tile_kernel<double, 16>), dim3(ntiles), dim3(kBlock), lds, s, a);
    else hipLaunchKernelGGL((assign_tile_kernel<float, 16>), dim3(ntiles), dim3(kBlock), lds, s, a);
  } else {
    if (f64) hipLaunchKernelGGL((assign_tile_kernel<double, kMaxCh>), dim3(ntiles), dim3(kBlock), lds, s, a);
    else hipLaunchKernelGGL((assign_tile_kernel<float, kMaxCh>), dim3(ntiles), dim3(kBlock), lds, s, a);
  }
  if (!P.box_mode) {
    const double vc = P.L * P.L * P.L / ((double)P.N * P.N * P.N);
    hipLaunchKernelGGL(norm_final_kernel, dim3(1), dim3(kBlock), 0, s, (const double*)P.d_sum_partials,
                       ntiles, P.d_scal, vc);
  }
  prof_end(P, kStAssign, s);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
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
