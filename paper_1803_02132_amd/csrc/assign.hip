// Weights, y-weighted density channels and mass assignment (Sec. 4.1, eq. 34;
// Sec. 4.2, eq. 39; Sec. 5.2, eq. 54).
//
// Assignment is a gather over tiles: particles are bucketed by the T^3 tile of
// their cell and by which neighbouring tiles their stencils reach, and one
// workgroup per output tile scatters into LDS the particles of its own tile
// and those of its 26 neighbours that reach it. Contributions are rounded to
// fixed point and added with integer LDS atomics, so every grid value is
// independent of thread and bucket order: the result is bitwise reproducible.
// One 64-bit word per channel at a plan-wide scale 2^e, with sum|w| 2^e below
// 2^61 (FP64 plans) or 2^51 (FP32 plans); in FP32 plans, tiles that run as a
// single work item instead add the two channels of a complex grid into one
// word as two 32-bit sums at a per-tile scale (half the atomics). Rounding to
// the nearest step is biased at that coarse step (many contributions are a
// fraction of it, and their fractional parts are not uniform), by about 1% of
// a step per contribution. A box plan's dn only scales by it; a survey's dn is
// the small difference of two window-shaped fields (galaxies and alpha
// randoms), where a relative bias of 1e-7 between the two already shows at
// the lowest k. Survey plans therefore round each packed contribution up with
// probability equal to its fractional part, the uniform variate a hash of the
// particle's stencil parameters and the node (deterministic, so results stay
// bitwise reproducible): unbiased to 2^-24 of a step. The survey randoms
// channel, which feeds the normalisation, always keeps its own word at the
// plan-wide scale.
#include <cmath>

#include "fft_reg.h"
#include "serve_policy.h"
#include "tsb_internal.h"

namespace tsb {

namespace {

constexpr int kMaxCh = 48;       // real channels (+1 randoms channel in survey mode)
constexpr int kMaxGrids = 32;
constexpr int kPrepBlocks = 512;

struct CatPtrs {
  const float *x, *y, *z, *w, *nbar;
  int64_t n;
  int wpow;   // 1: the weight w; 2: w^2 (the w^2-weighted fields N_L^M of the shot noise)
};

// The catalogue as the kernels read it; the plan's pass decides the weight power.
CatPtrs cat_ptrs(const Plan& P, const tsb_catalog* c) {
  CatPtrs p{};
  if (c) {
    p.x = c->x; p.y = c->y; p.z = c->z; p.w = c->w; p.nbar = c->nbar; p.n = c->n;
  }
  p.wpow = P.wpass ? 2 : 1;
  return p;
}

// The scalars of the plan's current pass: the measurement's own, or those of
// the w^2-weighted pass (its fixed-point scale; its alpha is -alpha^2, so that
// randoms enter the N fields with +alpha^2 w^2, eq. 46).
DevScalars* pass_scalars(const Plan& P) { return P.wpass ? P.d_scal_n : P.d_scal; }

__device__ inline double particle_weight(const CatPtrs& c, int64_t i, double P0) {
  double w = c.w ? (double)c.w[i] : 1.0;
  if (c.nbar && P0 > 0.0) w = w / (1.0 + (double)c.nbar[i] * P0);   // Sec. 5.2, eq. 54
  return c.wpow == 2 ? w * w : w;
}

// ----------------------------------------------------------------------------
// weights: sums, alpha, fixed-point scale, input validation

struct PrepArgs {
  CatPtrs d, r;
  double P0, inv_h, origin[3], obs[3];
  int N, box_mode, local;
  DevScalars* scal;
  double* partials;   // [gridDim][kPrepVals]
};

// Per-block reduction of the weights: sum w and sum |w| of data and randoms,
// then max |w| of data and randoms.
constexpr int kPrepVals = 6;

__device__ inline void block_reduce_prep(double* v, double* sh) {
  // fixed-order tree over the block
  const int t = threadIdx.x;
  for (int k = 0; k < kPrepVals; ++k) sh[k * kBlock + t] = v[k];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (t < s) {
      for (int k = 0; k < 4; ++k) sh[k * kBlock + t] += sh[k * kBlock + t + s];
      for (int k = 4; k < kPrepVals; ++k) sh[k * kBlock + t] = fmax(sh[k * kBlock + t], sh[k * kBlock + t + s]);
    }
    __syncthreads();
  }
  for (int k = 0; k < kPrepVals; ++k) v[k] = sh[k * kBlock];
}

__global__ void __launch_bounds__(kBlock) prep_kernel(PrepArgs a) {
  __shared__ double sh[kPrepVals * kBlock];
  double v[kPrepVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
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
      v[5] = fmax(v[5], fabs(w));
    } else {
      v[0] += w;
      v[2] += fabs(w);
      v[4] = fmax(v[4], fabs(w));
    }
  }
  if (err) atomicOr(&a.scal->err, err);
  block_reduce_prep(v, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < kPrepVals; ++k) a.partials[blockIdx.x * kPrepVals + k] = v[k];
}

__global__ void __launch_bounds__(kBlock) prep_final_kernel(const double* partials, int nblocks,
                                                            DevScalars* scal, int box_mode,
                                                            double n3, double volume, int fixed_bits,
                                                            const DevScalars* main) {
  __shared__ double sh[kPrepVals * kBlock];
  double v[kPrepVals] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += kBlock) {
    for (int k = 0; k < 4; ++k) v[k] += partials[b * kPrepVals + k];
    for (int k = 4; k < kPrepVals; ++k) v[k] = fmax(v[k], partials[b * kPrepVals + k]);
  }
  block_reduce_prep(v, sh);
  if (threadIdx.x == 0) {
    scal->sum_w = v[0];
    scal->sum_w_ran = v[1];
    scal->sum_abs = v[2];
    scal->sum_abs_ran = v[3];
    double alpha = box_mode ? 0.0 : (v[1] != 0.0 ? v[0] / v[1] : 0.0);   // Sec. 4.1
    if (main) alpha = -main->alpha * main->alpha;   // w^2 pass: randoms carry +alpha^2 (eq. 46)
    scal->alpha = alpha;
    // |y_L^M| <= 1 (Racah normalisation), so |c| <= max |w| (data) and
    // |alpha| max |w| (randoms)
    scal->cmax = fmax(v[4], fabs(alpha) * v[5]);
    const double wtot = v[2] + fabs(alpha) * v[3];
    int e = 40;
    if (wtot > 0.0 && isfinite(wtot)) {
      int ex;
      frexp(wtot, &ex);   // wtot < 2^ex
      e = fixed_bits - ex;
      if (e > 200) e = 200;
      if (e < -200) e = -200;
    }
    scal->scale = ldexp(1.0, e);
    scal->inv_scale = ldexp(1.0, -e);
    scal->mean_cell = box_mode && !main ? v[0] / n3 : 0.0;   // the N fields have no mean term
    scal->I = box_mode ? v[0] * v[0] * v[0] / (volume * volume) : 0.0;   // Sec. 4.4
  }
}

// ----------------------------------------------------------------------------
// bucketing by (tile, reach class)
//
// Over both grid copies a particle in cell c touches the nodes [c + lo, c + hi]
// of each axis (lo >= -1, hi <= 3). Per axis its class is 0 when that span
// leaves its tile downwards, 2 when it leaves upwards and 1 otherwise; the
// bucket key is tile * 27 + (9 cx + 3 cy + cz). A tile then reads, of each
// neighbour, only the classes that reach into it (about 2.5 tiles' worth of
// particles instead of 27).

constexpr int kClasses = 27;

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

struct BucketArgs {
  CatPtrs d, r;
  double inv_h, origin[3], P0;
  int N, T, NT, p, copies, box_mode;
  int colmode;        // 1: keys of the (x, y) columns of the column assignment
  int* count;         // [nbk]
  const int* start;   // [nbk + 1]
  int* keys;          // [particles] offset of each particle inside its bucket
};

// Grid coordinate (wrapped into [0, N) in box mode) and weight of particle i
// of the concatenated data + randoms list; false when it takes no part
// (non-finite input, or outside the grid in survey mode: both reported by the
// weight pass).
__device__ inline bool particle_u(const BucketArgs& a, int64_t i, double* u, double* w, bool* ran) {
  *ran = i >= a.d.n;
  const CatPtrs& c = *ran ? a.r : a.d;
  const int64_t j = *ran ? i - a.d.n : i;
  const double x[3] = {c.x[j], c.y[j], c.z[j]};
  *w = particle_weight(c, j, a.P0);
  bool ok = isfinite(*w);
  for (int ax = 0; ax < 3; ++ax) {
    u[ax] = (x[ax] - a.origin[ax]) * a.inv_h;
    if (!isfinite(u[ax])) {
      ok = false;
      continue;
    }
    if (u[ax] < 0.0 || u[ax] >= a.N) {
      if (!a.box_mode) {
        ok = false;
      } else {
        u[ax] = fmod(u[ax], (double)a.N);      // exact
        if (u[ax] < 0.0) u[ax] += a.N;
        if (u[ax] >= a.N) u[ax] -= a.N;        // -tiny + N rounds to N: the same point as 0
      }
    }
  }
  return ok;
}

// Bucket key of a particle that takes part (u in [0, N)).
__device__ inline int bucket_key(const BucketArgs& a, const double* u) {
  int tile = 0, cls = 0;
  for (int ax = 0; ax < 3; ++ax) {
    const int c = (int)floor(u[ax]);
    const int l = c % a.T;
    int lo = 1 << 30, hi = -(1 << 30);
    for (int g = 0; g < a.copies; ++g) {
      double wt[3];
      const int j0 = axis_stencil(u[ax] + 0.5 * g, a.p, wt);
      lo = min(lo, j0);
      hi = max(hi, j0 + a.p - 1);
    }
    const int k = (l + lo - c < 0) ? 0 : (l + hi - c >= a.T ? 2 : 1);
    tile = tile * a.NT + c / a.T;
    cls = cls * 3 + k;
  }
  return tile * kClasses + cls;
}

// Columns of the column assignment: kColW x kColW nodes in (x, y), all N in
// z. A particle is bucketed by the column of its lowest stencil node (over
// both grid copies) on each of x and y, and by how many columns up its
// stencil reaches there (0, 1 or 2: a stencil spans at most four nodes).
constexpr int kColW = 2;
constexpr int kColClasses = 9;

__device__ inline int column_key(const BucketArgs& a, const double* u) {
  const int NC = a.N / kColW;
  int col = 0, cls = 0;
  for (int ax = 0; ax < 2; ++ax) {
    int lo = 1 << 30, hi = -(1 << 30);
    for (int g = 0; g < a.copies; ++g) {
      double wt[3];
      const int j0 = axis_stencil(u[ax] + 0.5 * g, a.p, wt);
      lo = min(lo, j0);
      hi = max(hi, j0 + a.p - 1);
    }
    int lw = lo % a.N;
    if (lw < 0) lw += a.N;
    const int hc = lw / kColW;
    col = col * NC + hc;
    cls = cls * 3 + (lw - hc * kColW + hi - lo) / kColW;
  }
  return col * kColClasses + cls;
}

// Wavefront runs of equal keys: lanes holding the same key in a row take one
// atomic between them (catalogues are often stored in spatial order).
__device__ inline int run_end(unsigned long long heads, int lane) {
  const unsigned long long later = lane == 63 ? 0ull : (heads >> (lane + 1)) << (lane + 1);
  return later ? __ffsll((unsigned long long)later) - 1 : 64;
}

__device__ inline int run_head(unsigned long long heads, int lane) {
  const unsigned long long upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
  return 63 - __clzll((long long)(heads & upto));
}

// Bucket key of particle i (one that takes no part goes to a fixed bucket).
__device__ inline int particle_key(const BucketArgs& a, int64_t i) {
  double u[3], w;
  bool ran;
  if (a.colmode) return particle_u(a, i, u, &w, &ran) ? column_key(a, u) : 0;   // column 0, class 0
  return particle_u(a, i, u, &w, &ran) ? bucket_key(a, u) : kClasses / 2;       // tile 0, middle class
}

// Counts per bucket; each particle keeps its offset inside its bucket (in
// keys[]), so the fill needs no atomics: a run of equal keys in a wavefront
// takes one atomic, whose old value its lanes extend.
__global__ void __launch_bounds__(kBlock) bucket_count_kernel(BucketArgs a) {
  const int64_t ntot = a.d.n + a.r.n;
  const int lane = threadIdx.x & 63;
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < ntot; base += (int64_t)gridDim.x * kBlock) {
    const int64_t i = base + threadIdx.x;
    const int key = i < ntot ? particle_key(a, i) : -1;
    const int prev = __shfl_up(key, 1);
    const bool head = lane == 0 || key != prev;
    const unsigned long long heads = __ballot(head);
    int off = 0;
    if (head && key >= 0) off = atomicAdd(&a.count[key], run_end(heads, lane) - lane);
    const int hl = run_head(heads, lane);
    off = __shfl(off, hl) + (lane - hl);
    if (i < ntot) a.keys[i] = off;
  }
}

// Exclusive prefix sums of n ints (out has n + 1 entries): workgroup sums,
// a scan of those, then the per-workgroup scans.

__device__ inline int block_exclusive(int v, int* sh, int* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const int x = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  *total = sh[kBlock - 1];
  const int r = sh[t] - v;
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kBlock) scan_sums_kernel(const int* in, int64_t n, int* part) {
  __shared__ int sh[kBlock];
  const int64_t b0 = (int64_t)blockIdx.x * kScanChunk;
  int s = 0;
  for (int k = 0; k < kScanPer; ++k) {
    const int64_t i = b0 + (int64_t)k * kBlock + threadIdx.x;
    if (i < n) s += in[i];
  }
  int total;
  block_exclusive(s, sh, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kBlock) scan_parts_kernel(int* part, int nparts) {
  __shared__ int sh[kBlock];
  int carry = 0;
  for (int b0 = 0; b0 < nparts; b0 += kBlock) {
    const int i = b0 + threadIdx.x;
    const int v = i < nparts ? part[i] : 0;
    int total;
    const int e = block_exclusive(v, sh, &total);
    if (i < nparts) part[i] = carry + e;
    carry += total;
  }
}

__global__ void __launch_bounds__(kBlock) scan_out_kernel(const int* in, int64_t n, const int* part, int* out) {
  __shared__ int sh[kBlock];
  const int64_t b0 = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
  int v[kScanPer];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = b0 + k < n ? in[b0 + k] : 0;
    s += v[k];
  }
  int total;
  int run = part[blockIdx.x] + block_exclusive(s, sh, &total);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int64_t i = b0 + k;
    if (i < n) out[i] = run;
    run += v[k];
    if (i == n - 1) out[n] = run;
  }
  if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
}


// Channel layout shared by the record and tile kernels.
struct ChanInfo {
  int nch;                     // real channels (the survey randoms channel is nch)
  int local;
  int window;                  // window multipoles: randoms +alpha, galaxies 0 (Sec. 6.1, eq. 58)
  double obs[3];
  int chL[kMaxCh], chM[kMaxCh], chPart[kMaxCh];
  double ynorm[45];
};

template <int NCH>
__device__ inline void channel_values(const ChanInfo& ci, double x, double y, double z, double w, bool ran,
                                      double alpha, double* cv) {
  // c = w y_L^M*(x^) (eq. 34); randoms carry -alpha (eq. 34), or for the window
  // multipoles +alpha with the galaxies left out; survey mode adds
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
  const double s = ci.window ? (ran ? alpha * w : 0.0) : (ran ? -alpha * w : w);
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

// Survey plans store each channel weight in FP32 by rounding up or down with
// probability given by the distance to the two neighbouring FP32 values (the
// uniform variate a hash of the particle's catalogue index and the channel),
// so that weights shared by many particles (n-bar takes few values) carry no
// common rounding error into the cancellation of galaxies against randoms.
__device__ inline unsigned wmix32(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

__device__ inline float stochastic_f32(double x, unsigned h) {
  const float f = (float)x;
  if ((double)f == x || !isfinite(f)) return f;
  const float lo = (double)f < x ? f : nextafterf(f, -INFINITY);
  const float hi = (double)f < x ? nextafterf(f, INFINITY) : f;
  const double pr = (x - (double)lo) / ((double)hi - (double)lo);
  return (double)h * 2.3283064365386963e-10 < pr ? hi : lo;   // h 2^-32
}

// Particle records in bucket order, one contiguous record each: the grid
// coordinate u (3 FP64; NaN in u_x marks a particle that takes no part), then
// its channel weights in the plan precision in slot order: slots 2g and 2g+1
// hold the real and imaginary channel of complex grid g (0 where grid g has no
// imaginary channel), and in survey mode slot 2 ngrid the randoms channel;
// stride a multiple of 16 bytes.
template <typename T>
struct Records {
  char* base;
  int stride;
  int64_t cap;
  __device__ double* u(int64_t slot) const { return (double*)(base + slot * stride); }
  __device__ T* c(int64_t slot) const { return (T*)(base + slot * stride + 24); }
};

template <typename T, int NCH>
struct FillArgs {
  BucketArgs b;
  ChanInfo ci;
  Records<T> rec;
  int nchx;
  int slot_of[kMaxCh];   // channel -> record slot
  int zslot;             // slot that stays 0 (a grid without imaginary channel), or -1
  const DevScalars* scal;
};

template <typename T, int NCH>
__global__ void __launch_bounds__(kBlock) bucket_fill_kernel(FillArgs<T, NCH> a) {
  const int64_t ntot = a.b.d.n + a.b.r.n;
  const double alpha = a.scal->alpha;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < ntot; i += (int64_t)gridDim.x * kBlock) {
    double u[3], w;
    bool ran;
    const bool ok = particle_u(a.b, i, u, &w, &ran);
    // the key again (as particle_key forms it) and the offset the count kept
    const int key = ok ? (a.b.colmode ? column_key(a.b, u) : bucket_key(a.b, u)) : (a.b.colmode ? 0 : kClasses / 2);
    const int64_t slot = (int64_t)a.b.start[key] + a.b.keys[i];
    const CatPtrs& c = ran ? a.b.r : a.b.d;
    const int64_t j = ran ? i - a.b.d.n : i;
    double* ru = a.rec.u(slot);
    ru[0] = ok ? u[0] : NAN;
    ru[1] = u[1];
    ru[2] = u[2];
    double cv[NCH];
    channel_values<NCH>(a.ci, c.x[j], c.y[j], c.z[j], ok ? w : 0.0, ran, alpha, cv);
    // the w^2 pass builds no normalisation: its randoms channel stays empty
    if (a.b.d.wpow == 2 && a.ci.nch < NCH) cv[a.ci.nch] = 0.0;
    T* rc = a.rec.c(slot);
    if (sizeof(T) == 4 && !a.b.box_mode) {
      const unsigned pk = wmix32((unsigned)i * 0x9E3779B9U ^ (unsigned)(i >> 32));
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
        if (ch < a.nchx) rc[a.slot_of[ch]] = (T)stochastic_f32(cv[ch], wmix32(pk + (unsigned)ch * 0x85EBCA6BU));
    } else {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
        if (ch < a.nchx) rc[a.slot_of[ch]] = (T)cv[ch];
    }
    if (a.zslot >= 0) rc[a.zslot] = (T)0;
  }
}

// ----------------------------------------------------------------------------
// tile assignment

constexpr int kMaxRanges = 64;

struct TileArgs {
  double inv_h, h, origin[3];
  int N, T, NT, p, copies, box_mode;
  int lt;                      // log2 T (T is 4 or 8)
  ChanInfo ci;
  int ngrid;                   // complex output grids (record slots 2g, 2g+1)
  int nw;                      // 64-bit fixed-point words per node
  double wmax;                 // largest node weight of the kernel (p = 3: 0.75^3)
  int wr;                      // word of the survey randoms channel, or -1
  const int* start;            // bucket starts [ntiles * 27 + 1]
  const DevScalars* scal;
  void* out;                   // [copies][ngrid][N^3] complex
  double* tile_I;              // survey: per-tile sum of (alpha R)^3
  // reads of one tile: neighbour offset (9 (dx+1) + 3 (dy+1) + dz + 1) and class range
  int nr;
  int rd[kMaxRanges], rcl[kMaxRanges], rch[kMaxRanges];
  // work items: the extra parts of split tiles (a tile with more than
  // part_visits visits), then part 0 of every tile
  const int2* work;            // extra parts (tile, part >= 1)
  const int* nextra;           // number of extra parts (device)
  int ntiles;
  const int* hslot;            // per tile: heavy slot or -1
  unsigned long long* heavy;   // [slot][copies][nw][T^3] fixed-point sums of split tiles
  int max_heavy;               // slots of split tiles
};

// Ranges of one tile (wave-parallel): start and length of range r of tile t.
__device__ inline void tile_range(const TileArgs& a, int tile, int r, int* st, int* len) {
  const int NT = a.NT;
  const int tx = tile / (NT * NT), ty = (tile / NT) % NT, tz = tile % NT;
  const int d = a.rd[r];
  const int nx = (tx + d / 9 - 1 + NT) % NT, ny = (ty + (d / 3) % 3 - 1 + NT) % NT, nz = (tz + d % 3 - 1 + NT) % NT;
  const int64_t nt = ((int64_t)nx * NT + ny) * NT + nz;
  *st = a.start[nt * kClasses + a.rcl[r]];
  *len = a.start[nt * kClasses + a.rch[r]] - *st;
}


// Node position (relative to the observer) of grid copy g, and y_L^M*(x^) of
// real channel ch there (global LOS: 1). The box-mode subtraction of the mean
// (Sec. 4.4) is this times sum w / N^3; it is applied to the spectra.
__device__ inline double node_y(const ChanInfo& ci, int ch, double ux, double uy, double uz) {
  double re = 1.0, im = 0.0;
  if (ci.local) ylm_pos_m(ci.chL[ch], ci.chM[ch], ux, uy, uz, ci.ynorm, &re, &im);
  return ci.chPart[ch] ? -im : re;
}

__device__ inline void node_dir(const double* origin, double h, const double* obs, int ix, int iy, int iz, int g,
                                double* u) {
  const double px = origin[0] + (ix - 0.5 * g) * h - obs[0];
  const double py = origin[1] + (iy - 0.5 * g) * h - obs[1];
  const double pz = origin[2] + (iz - 0.5 * g) * h - obs[2];
  const double r = sqrt(px * px + py * py + pz * pz);
  u[0] = 0.0;
  u[1] = 0.0;
  u[2] = 1.0;
  if (r > 0.0) {
    u[0] = px / r;
    u[1] = py / r;
    u[2] = pz / r;
  }
}

constexpr int kVisitChunk = 128;  // particles staged in LDS at a time (a power of two)
// Visits per work item; busier tiles are split. A packed FP32 item's
// fixed-point step grows with its visits: box plans take 512 (half the slots
// and slot atomics of 256), survey plans, whose density is the small
// difference of two window-shaped fields and whose packed contributions are
// rounded stochastically, keep 256 (one more fraction bit).
constexpr int kPartVisits = 256;
constexpr int kPartVisitsBox = 512;
__host__ __device__ inline int part_visits(int box_mode) { return box_mode ? kPartVisitsBox : kPartVisits; }
constexpr int kTileBlock = 256;    // threads per workgroup of the tile kernel
constexpr int kMinHeavy = 2048;   // split-tile slots at least (or one per tile); others run whole

// A staged (particle, grid copy) visit: per axis the stencil parameter d (the
// kernel weights are functions of d and the stencil index) and which stencil
// nodes fall inside the tile: the first in-tile stencil index s0, their count
// and the in-tile node of each stencil index (consecutive stencil indices;
// with one tile per axis the nodes may wrap inside the tile). The channel
// weights live per particle beside it. A work item is one (visit, in-tile x
// node): it adds the particle's contributions to the in-tile (y, z) nodes of
// that plane.
template <typename T>
struct Visit {
  T d[3];
  unsigned char s0[3], cnt[3], l[3][3];
};

// Weights of the p stencil nodes of the order-p kernel at parameter d (the
// same expressions as axis_stencil; unused entries 0).
template <typename T>
__device__ inline void stencil_weights(int p, T d, T* w) {
  const T h = (T)0.5;
  if (p == 3) {
    w[0] = h * (h - d) * (h - d);
    w[1] = (T)0.75 - d * d;
    w[2] = h * (h + d) * (h + d);
  } else if (p == 2) {
    w[0] = (T)1 - d;
    w[1] = d;
    w[2] = (T)0;
  } else {
    w[0] = (T)1;
    w[1] = (T)0;
    w[2] = (T)0;
  }
}

// w[s] for a stencil index s in 0..2 held in a register (static indexing)
template <typename T>
__device__ inline T pick3(const T* w, int s) {
  return s == 0 ? w[0] : (s == 1 ? w[1] : w[2]);
}

// Parameter d of axis_stencil for grid coordinate u (the weights follow from
// stencil_weight): TSC and NGP measure from the nearest node, CIC from the
// node below.
__device__ inline double stencil_param(double u, int p, int* j0) {
  if (p == 2) {
    const double j = floor(u);
    *j0 = (int)j;
    return u - j;
  }
  const double j = floor(u + 0.5);
  *j0 = (int)j - (p == 3 ? 1 : 0);
  return u - j;
}

// A 32-bit mix with full avalanche (two multiply-xorshift rounds).
__device__ inline unsigned mix32(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

// floor(x) + 1 with probability frac(x) given a uniform u in [0, 1): the
// expectation is x (frac(x) = x - floor(x) is exact in FP32).
__device__ inline int dither_round(float x, float u) {
  const float f = floorf(x);
  return (int)f + ((x - f) > u ? 1 : 0);
}

// Fixed-point rounding to the nearest integer. FP64 plans: llrint. FP32 plans:
// |x| < 2^51, so adding 1.5 * 2^52 leaves round-to-nearest(x) in the low
// mantissa bits (exact).
template <typename T>
__device__ inline long long to_fixed(double x) {
  if constexpr (sizeof(T) == 4) {
    return __double_as_longlong(x + 6755399441055744.0) - 0x4338000000000000LL;
  } else {
    return llrint(x);
  }
}

// Packed FP32 tiles add the two channels of a complex grid in one 64-bit
// word: word = hi 2^32 + lo (two's complement, modulo 2^64), with both sums
// below 2^31 in magnitude, so each is recovered exactly from the total. The
// low dword is lo, the high dword hi - 1 when lo < 0.
__device__ inline unsigned long long pack2(int lo, int hi) {
  return ((unsigned long long)(unsigned)(hi + (lo >> 31)) << 32) | (unsigned)lo;
}

__device__ inline void unpack2(unsigned long long v, int* lo, int* hi) {
  *lo = (int)(unsigned)v;
  *hi = (int)(unsigned)(v >> 32) - (*lo >> 31);
}

// Exponent of the per-tile fixed-point scale of packed FP32 tiles: each
// half-word sum is bounded by (visits of the tile) * max |c| * (largest node
// weight of the kernel), and the scale maps that bound below 2^30. A
// contribution is the FP32 product c W 2^e rounded to the nearest integer
// (ties to even), so the rounding errors carry no bias. Packing is used for
// work items of at most part_visits visits (a whole tile, or a part of a
// split one), so the fixed-point step is at most 2^-21 max |c| W_max.
__device__ inline int tile_exponent(int visits, double cw) {
  const double bound = (double)visits * cw;
  if (!(bound > 0.0) || !isfinite(bound)) return 0;
  int ex;
  frexp(bound, &ex);   // bound < 2^ex
  return min(100, max(-100, 30 - ex));
}

// A grid value that this kernel never reads back: streamed past the caches
// (nontemporal store) for FP32, a plain store for FP64.
template <typename T>
__device__ inline void store_stream(typename cplx<T>::type* p, typename cplx<T>::type v) {
  if constexpr (sizeof(T) == 4) {
    unsigned long long bits;
    __builtin_memcpy(&bits, &v, 8);
    __builtin_nontemporal_store(bits, (unsigned long long*)p);
  } else {
    *p = v;
  }
}

// One grid copy's fixed-point words of a node -> the complex output grids:
// packed (word g holds grid g, tile scale) or one word per channel slot
// (words 2g and 2g+1, plan-wide scale). With clear, the words read are set
// to zero (the accumulators then start the next work item cleared).
template <typename T, bool clear>
__device__ inline void put_node(unsigned long long* w, size_t wstride, int ngrid, bool packed, int et_neg,
                                double inv_scale, typename cplx<T>::type* out, size_t gstride) {
  typedef typename cplx<T>::type T2;
  for (int gr = 0; gr < ngrid; ++gr) {
    T2 o;
    if (packed) {
      int lo, hi;
      unpack2(w[(size_t)gr * wstride], &lo, &hi);
      o.x = (T)ldexpf((float)lo, et_neg);
      o.y = (T)ldexpf((float)hi, et_neg);
      if (clear) w[(size_t)gr * wstride] = 0ull;
    } else {
      o.x = (T)((double)(long long)w[(size_t)(2 * gr) * wstride] * inv_scale);
      o.y = (T)((double)(long long)w[(size_t)(2 * gr + 1) * wstride] * inv_scale);
      if (clear) w[(size_t)(2 * gr) * wstride] = w[(size_t)(2 * gr + 1) * wstride] = 0ull;
    }
    store_stream<T>(out + (size_t)gr * gstride, o);
  }
}

// Persistent workgroups walk the work items (a tile, or a part of a busy
// tile). The particles that reach the tile are staged 128 at a time as visits
// (stencil parameters and in-tile node ranges computed once per particle and
// grid copy); then every (visit, in-tile x node) is one work item over all
// lanes, which adds the particle's fixed-point contributions to each in-tile
// (y, z) node of that plane and every channel. Packed FP32 items (a whole
// tile or a part of a split one) stage both grid copies in one pass (their
// two-channel words of both copies fit the LDS of one unpacked copy); other
// items run one copy per pass. Parts of split tiles add their sums into the
// tile's slot; whole tiles write their nodes out. FP32 plans with up to 8
// channel slots keep four workgroups per CU.
template <typename T, int NCH>
__global__ void __launch_bounds__(kTileBlock, (sizeof(T) == 4 && NCH <= 8) ? 4 : 1)
    assign_tile_kernel(TileArgs a, Records<T> rec) {
  typedef typename cplx<T>::type T2;
  constexpr int kPC = sizeof(T) == 4 ? 2 : 1;   // grid copies staged per pass at most
  constexpr int kV = kVisitChunk * kPC;         // visits per chunk
  extern __shared__ unsigned long long acc[];   // [nw][T^3]
  __shared__ int r_start[2][kMaxRanges];        // range tables of the current and the next work item
  __shared__ int r_off[2][kMaxRanges + 1];
  __shared__ int item[2][3];                    // tile, part, heavy slot
  __shared__ int r_code[kMaxRanges];            // neighbour offset | low class << 8 | high class << 16
  __shared__ Visit<T> vis[kV];                  // [copy in pass][particle]
  __shared__ T pch[kVisitChunk][NCH];           // channel weights per staged particle
  __shared__ int it_first[kV];                  // first work item of each visit
  __shared__ int wtot[kTileBlock / 64];         // items of each staging wavefront
  __shared__ double wsum[kTileBlock / 64];
  __shared__ unsigned char it_vis[kV * 3];
  const int TS = a.T, T3 = TS * TS * TS;
  const int npair = a.ngrid, nw = a.nw, wr = a.wr;
  const int nslot = 2 * npair;   // grid slots; the randoms slot sits in register NCH - 1
  const int nextra = *a.nextra, nwork = a.ntiles + nextra;
  const int N = a.N, p = a.p;
  const int NT = a.NT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int vt = threadIdx.x & (kVisitChunk - 1);   // the particle this thread stages and prefetches
  T2* out = (T2*)a.out;
  const size_t N3 = (size_t)N * N * N;
  const double scale = a.scal->scale, inv_scale = a.scal->inv_scale, cmax = a.scal->cmax, alpha = a.scal->alpha;
  const int part_v = part_visits(a.box_mode);

  // Work-item pipeline: the ranges of the next-but-one item are fetched into
  // the first wavefront's registers, and the first chunk of particle records
  // of the next item into registers (each particle in every thread that
  // stages it), while the current item is processed.
  // The loads of a fetch stay in flight until the item is published one work
  // item later: the neighbour ranges sit in LDS for the whole kernel,
  // ordinary items need no load to name their tile, and a range's length is
  // formed only at publication.
  if (threadIdx.x < kMaxRanges) {
    const int r = (int)threadIdx.x < a.nr ? (int)threadIdx.x : 0;
    r_code[threadIdx.x] = a.rd[r] | a.rcl[r] << 8 | a.rch[r] << 16;
  }
  // the accumulators start cleared; afterwards every pass's write-out clears
  // the words it reads
  for (int i = threadIdx.x; i < nw * T3; i += kTileBlock) acc[i] = 0ull;
  __syncthreads();
  int pf_tile = 0, pf_hs = -1, pf_part = 0, pf_st = 0, pf_en = 0;
  auto fetch = [&](int w) {
    if (threadIdx.x < 64 && w < nwork) {
      int t = w - nextra, part = 0;
      if (w < nextra) {
        const int2 wk = a.work[w];
        t = wk.x;
        part = wk.y;
      }
      pf_tile = t;
      pf_part = part;
      pf_hs = a.hslot[t];
      // every lane loads (lanes past the ranges repeat range 0 and are
      // masked at publication), so no register is cleared under a load
      const int code = r_code[lane], my_d = code & 255, my_lo = (code >> 8) & 255, my_hi = code >> 16;
      const int tx = t / (NT * NT), ty = (t / NT) % NT, tz = t % NT;
      const int nx = (tx + my_d / 9 - 1 + NT) % NT, ny = (ty + (my_d / 3) % 3 - 1 + NT) % NT,
                nz = (tz + my_d % 3 - 1 + NT) % NT;
      const int64_t nt = ((int64_t)nx * NT + ny) * NT + nz;
      pf_st = a.start[nt * kClasses + my_lo];
      pf_en = a.start[nt * kClasses + my_hi];
    }
  };
  auto publish = [&](int b) {   // the fetched item -> range table b (first wavefront)
    if (threadIdx.x < 64) {
      int inc = lane < a.nr ? pf_en - pf_st : 0;
      for (int off = 1; off < 64; off <<= 1) {
        const int x = __shfl_up(inc, off);
        if (lane >= off) inc += x;
      }
      r_start[b][lane] = pf_st;
      r_off[b][lane + 1] = inc;
      if (lane == 0) {
        r_off[b][0] = 0;
        item[b][0] = pf_tile;
        item[b][1] = pf_part;
        item[b][2] = pf_hs;
      }
    }
  };
  auto window = [&](int b, int* v0, int* v1) {   // visits of the item in table b
    const int total = r_off[b][64], hs = item[b][2];
    *v0 = hs >= 0 ? item[b][1] * part_v : 0;
    *v1 = hs >= 0 ? min(total, *v0 + part_v) : total;
  };
  auto load_rec = [&](int b, int idx, double* u, T* cv) {   // visit idx of table b
    int lo = 0, hi = a.nr;   // r_off[lo] <= idx < r_off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (r_off[b][mid] <= idx) lo = mid;
      else hi = mid;
    }
    const int64_t slot = r_start[b][lo] + (idx - r_off[b][lo]);
    const double* ru = rec.u(slot);
    u[0] = ru[0];
    u[1] = ru[1];
    u[2] = ru[2];
    const T* rc = rec.c(slot);
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) cv[ch] = ch < nslot ? rc[ch] : (T)0;
    if (wr >= 0) cv[NCH - 1] = rc[nslot];
  };
  double cu[3] = {0.0, 0.0, 0.0}, nu[3] = {0.0, 0.0, 0.0};
  T cc[NCH], ncv[NCH];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) cc[ch] = ncv[ch] = (T)0;
  int cb = 0;
  if ((int)blockIdx.x < nwork) {
    fetch(blockIdx.x);
    publish(0);
    __syncthreads();
    {
      int v0, v1;
      window(0, &v0, &v1);
      if (v0 + vt < v1) load_rec(0, v0 + vt, cu, cc);
    }
    fetch(blockIdx.x + gridDim.x);
  }
  // the previous work item ended with a barrier after its last LDS use (and
  // published this item's table before one)
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
  const int tile = item[cb][0], hs = item[cb][2];   // hs >= 0: split tile, sums go to its slot
  const int tx = tile / (NT * NT), ty = (tile / NT) % NT, tz = tile % NT;
  const int o3[3] = {tx * TS, ty * TS, tz * TS};
  int v0, v1;
  window(cb, &v0, &v1);
  // FP32 work items of at most part_v visits pack two channels per word,
  // both grid copies in one pass (word of copy c, grid k: c * npair + k), at
  // a scale of their own: a whole tile (from its visits), or a part of a
  // split tile (from part_v, the same for every part: which part a
  // particle falls in depends on the bucket order, its rounding must not).
  // A part converts its sums to the plan's scale, exactly, when it adds them
  // into the slot (the shift plan_e - et is never negative then).
  const int plan_e = ilogb(scale);
  const int et_item = tile_exponent(hs >= 0 ? part_v : v1 - v0, cmax * a.wmax);
  const bool packed = sizeof(T) == 4 && (r_off[cb][64] <= part_v || (hs >= 0 && plan_e >= et_item));
  const unsigned tile_key = mix32((unsigned)tile * 0x9E3779B9U + 0x85EBCA6BU);
  const int et = packed ? et_item : 0;
  const float tscale = ldexpf(1.0f, et);
  const int ncp = packed ? a.copies : 1;                 // grid copies per pass
  const int wrw = wr < 0 ? -1 : (packed ? a.copies * npair : wr);   // randoms word
  const bool has_next = w + (int)gridDim.x < nwork;
  double sumI = 0.0;
  for (int g0 = 0; g0 < a.copies; g0 += ncp) {
    for (int c0 = v0; c0 < v1; c0 += kVisitChunk) {
      const int nv = min(kVisitChunk, v1 - c0);
      if (c0 != v0) __syncthreads();   // the previous chunk is consumed
      int items = 0;
      {
        // staging: thread t stages copy g0 + (t >> 7) of particle t & 127
        const int cp = threadIdx.x / kVisitChunk;
        if (cp < ncp && vt < nv) {
          double u[3];
          T cv[NCH];
          if (c0 == v0) {   // the item's first chunk: already in registers
            u[0] = cu[0];
            u[1] = cu[1];
            u[2] = cu[2];
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) cv[ch] = cc[ch];
          } else {
            load_rec(cb, c0 + vt, u, cv);
          }
          Visit<T>& V = vis[threadIdx.x];
          int cnt[3] = {0, 0, 0};
          if (isfinite(u[0])) {
            for (int ax = 0; ax < 3; ++ax) {
              int j0;
              V.d[ax] = (T)stencil_param(u[ax] + 0.5 * (g0 + cp), p, &j0);
              int s0 = -1;
              for (int sidx = 0; sidx < p; ++sidx) {
                int jj = j0 + sidx;
                jj += jj < 0 ? N : (jj >= N ? -N : 0);
                const int l = jj - o3[ax];
                const bool in = l >= 0 && l < TS;
                V.l[ax][sidx] = (unsigned char)(in ? l : 0);
                if (in) {
                  if (s0 < 0) s0 = sidx;
                  ++cnt[ax];
                }
              }
              V.s0[ax] = (unsigned char)max(s0, 0);
            }
          }
          if (cp == 0) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) pch[vt][ch] = cv[ch];
          }
          if (cnt[0] == 0 || cnt[1] == 0 || cnt[2] == 0) cnt[0] = cnt[1] = cnt[2] = 0;
          V.cnt[0] = (unsigned char)cnt[0];
          V.cnt[1] = (unsigned char)cnt[1];
          V.cnt[2] = (unsigned char)cnt[2];
          items = cnt[0];
        }
      }
      int inc = items;
      for (int off = 1; off < 64; off <<= 1) {
        const int x = __shfl_up(inc, off);
        if (lane >= off) inc += x;
      }
      if (lane == 63) wtot[wave] = inc;
      __syncthreads();
      int nitems = 0, wbase = 0;
#pragma unroll
      for (int k = 0; k < kTileBlock / 64; ++k) {
        wbase += k < wave ? wtot[k] : 0;
        nitems += wtot[k];
      }
      {
        // item -> visit map (visits of a pass are numbered by staging thread)
        const int first = wbase + inc - items;
        if (threadIdx.x < kV) it_first[threadIdx.x] = first;
        for (int k = 0; k < items; ++k) it_vis[first + k] = (unsigned char)threadIdx.x;
      }
      __syncthreads();
      // items in a scrambled order (multiplier prime to their number), so that
      // the lanes of a wavefront work on particles far apart in the chunk
      const int imult = nitems % 97 ? 97 : (nitems % 101 ? 101 : 103);
      for (int i0 = threadIdx.x; i0 < nitems; i0 += kTileBlock) {
        const int it = (i0 * imult) % nitems;
        const int vi = it_vis[it];
        const Visit<T>& V = vis[vi];
        const int cp = vi / kVisitChunk, pv = vi & (kVisitChunk - 1);
        // the particle's data to registers once (the atomics below may alias it)
        T c[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) c[ch] = pch[pv][ch];
        const int sx = it - it_first[vi];
        const int cy = V.cnt[1], cz = V.cnt[2];
        const int sx0 = V.s0[0] + sx, sy0 = V.s0[1], sz0 = V.s0[2];
        T wa[3], wb[3], wc[3];
        stencil_weights<T>(p, V.d[0], wa);
        stencil_weights<T>(p, V.d[1], wb);
        stencil_weights<T>(p, V.d[2], wc);
        const T wx = pick3(wa, sx0);
        const int ox = V.l[0][sx0] * TS * TS;
        T wy[3], wz[3];
        int oy[3], oz[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int ky = min(sy0 + k, 2), kz = min(sz0 + k, 2);   // indices past the count are not used
          wy[k] = pick3(wb, ky);
          oy[k] = V.l[1][ky] * TS;
          wz[k] = pick3(wc, kz);
          oz[k] = V.l[2][kz];
        }
        const T wxs = packed ? wx * (T)tscale : wx;   // packed: the tile scale folded into the x weight
        unsigned long long* cbase = acc + (packed ? (size_t)cp * npair * T3 : 0);
        const bool randoms = wrw >= 0 && g0 + cp == 0;
        // survey plans: the particle's key for the dithered rounding (its
        // stencil parameters of this copy, the tile, the copy)
        unsigned pkey = 0U;
        if (sizeof(T) == 4 && packed && !a.box_mode)
          pkey = mix32(__float_as_uint((float)V.d[0]) ^ mix32(__float_as_uint((float)V.d[1]) ^
                       mix32(__float_as_uint((float)V.d[2]) ^ tile_key)) ^ (unsigned)(g0 + cp));
#pragma unroll
        for (int sy = 0; sy < 3; ++sy) {
          if (sy >= cy) break;
          const T wxy = wxs * wy[sy];
          const int base = ox + oy[sy];
#pragma unroll
          for (int sz = 0; sz < 3; ++sz) {
            if (sz >= cz) break;
            const T Wt = wxy * wz[sz];
            unsigned long long* cellp = cbase + base + oz[sz];
            if (sizeof(T) == 4 && packed && !a.box_mode) {
              const unsigned h = mix32(pkey ^ (unsigned)(base + oz[sz]) * 0x9E3779B9U);
              const float u = (float)(h >> 8) * 5.9604644775390625e-8f;   // 2^-24
#pragma unroll
              for (int k = 0; k < NCH / 2; ++k) {
                if (k >= npair) break;
                atomicAdd(cellp + (size_t)k * T3, pack2(dither_round((float)c[2 * k] * (float)Wt, u),
                                                        dither_round((float)c[2 * k + 1] * (float)Wt, u)));
              }
            } else if (sizeof(T) == 4 && packed) {
#pragma unroll
              for (int k = 0; k < NCH / 2; ++k) {
                if (k >= npair) break;
                atomicAdd(cellp + (size_t)k * T3, pack2(__float2int_rn((float)c[2 * k] * (float)Wt),
                                                        __float2int_rn((float)c[2 * k + 1] * (float)Wt)));
              }
            } else {
              const double Ws = (double)Wt * scale;
#pragma unroll
              for (int k = 0; k < NCH; ++k) {
                if (k >= nslot) break;
                atomicAdd(cellp + (size_t)k * T3, (unsigned long long)to_fixed<T>((double)c[k] * Ws));
              }
            }
            if (randoms) {   // randoms channel: full 64-bit word, plan-wide scale
              const double Wr = (double)(wx * wy[sy] * wz[sz]) * scale;
              atomicAdd(acc + (size_t)wrw * T3 + base + oz[sz],
                        (unsigned long long)to_fixed<T>((double)c[NCH - 1] * Wr));
            }
          }
        }
      }
    }
    if (g0 == 0 && has_next) publish(cb ^ 1);
    __syncthreads();
    if (g0 == 0 && has_next) {
      // the next item's first chunk of records, then the ranges of the
      // next-but-one item, loaded while this one finishes
      int n0, n1;
      window(cb ^ 1, &n0, &n1);
      if (n0 + vt < n1) load_rec(cb ^ 1, n0 + vt, nu, ncv);
      fetch(w + 2 * gridDim.x);
    }
    if (hs >= 0) {
      // part of a split tile: add the fixed-point sums into its slot
      // (integer, order-free; the randoms word is the last one, copy 0 only)
      if (packed) {
        // both copies in this pass: each two-channel word unpacks into the
        // slot's channel words, shifted to the plan's scale (exact)
        const int sh = plan_e - et;
        for (int i = threadIdx.x; i < ncp * npair * T3; i += kTileBlock) {
          const unsigned long long v = acc[i];
          if (v == 0ull) continue;
          const int cell = i & (T3 - 1), ck = i / T3, q = ck / npair, k = ck - q * npair;
          unsigned long long* hb = a.heavy + ((size_t)hs * a.copies + g0 + q) * nw * T3 + cell;
          int lo, hi;
          unpack2(v, &lo, &hi);
          atomicAdd(hb + (size_t)(2 * k) * T3, (unsigned long long)lo << sh);
          atomicAdd(hb + (size_t)(2 * k + 1) * T3, (unsigned long long)hi << sh);
          acc[i] = 0ull;
        }
        if (wrw >= 0) {
          unsigned long long* hb = a.heavy + (size_t)hs * a.copies * nw * T3 + (size_t)wr * T3;
          for (int cell = threadIdx.x; cell < T3; cell += kTileBlock) {
            const unsigned long long v = acc[(size_t)wrw * T3 + cell];
            if (v == 0ull) continue;
            atomicAdd(hb + cell, v);
            acc[(size_t)wrw * T3 + cell] = 0ull;
          }
        }
      } else {
        const int nwg = (g0 == 0 || wr < 0) ? nw : nw - 1;
        unsigned long long* hb = a.heavy + ((size_t)hs * a.copies + g0) * nw * T3;
        for (int i = threadIdx.x; i < nwg * T3; i += kTileBlock) {
          const unsigned long long v = acc[i];
          if (v != 0ull) {
            atomicAdd(hb + i, v);
            acc[i] = 0ull;
          }
        }
      }
      __syncthreads();
      continue;
    }
    // write out the copies of this pass
    {
      const int lt = a.lt, tm = TS - 1;
      for (int cp = 0; cp < ncp; ++cp) {
        T2* tout = out + (size_t)(g0 + cp) * npair * N3 + ((size_t)o3[0] * N + o3[1]) * N + o3[2];
        unsigned long long* cw = acc + (packed ? (size_t)cp * npair * T3 : 0);
        for (int cell = threadIdx.x; cell < T3; cell += kTileBlock) {
          const int lx = cell >> (2 * lt), ly = (cell >> lt) & tm, lz = cell & tm;
          put_node<T, true>(cw + cell, T3, npair, packed, -et, inv_scale, tout + ((lx * N + ly) * N + lz), N3);
        }
      }
      if (wrw >= 0 && g0 == 0) {
        // Sec. 4.2, eq. 37: sum_j (alpha R_j)^3 over this tile
        for (int cell = threadIdx.x; cell < T3; cell += kTileBlock) {
          const double v = alpha * (double)(long long)acc[(size_t)wrw * T3 + cell] * inv_scale;
          acc[(size_t)wrw * T3 + cell] = 0ull;
          sumI += v * v * v;
        }
      }
    }
    __syncthreads();
  }
  if (wr >= 0 && hs < 0) {
    // fixed-order sum: within each wavefront, then over the wavefronts
    for (int off = 32; off > 0; off >>= 1) sumI += __shfl_xor(sumI, off);
    if (lane == 0) wsum[wave] = sumI;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int i = 0; i < kTileBlock / 64; ++i) t += wsum[i];
      a.tile_I[tile] = t;
    }
  }
  // advance the pipeline
  cb ^= 1;
  cu[0] = nu[0];
  cu[1] = nu[1];
  cu[2] = nu[2];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) cc[ch] = ncv[ch];
  }   // work items
}

// Split tiles (one word per channel slot, plan-wide scale): convert the
// summed fixed-point grids of each heavy slot, then clear the slot.
template <typename T>
__global__ void __launch_bounds__(kBlock) heavy_final_kernel(TileArgs a, const int* heavy_tile, const int* nheavy) {
  typedef typename cplx<T>::type T2;
  __shared__ double sh[kBlock];
  const int slot = blockIdx.x;
  if (slot >= min(*nheavy, a.max_heavy)) return;
  const int tile = heavy_tile[slot];
  const int TS = a.T, T3 = TS * TS * TS, N = a.N, NT = a.NT;
  const int nw = a.nw, wr = a.wr;
  const int o3[3] = {tile / (NT * NT) * TS, (tile / NT) % NT * TS, tile % NT * TS};
  const double inv_scale = a.scal->inv_scale;
  T2* out = (T2*)a.out;
  const size_t N3 = (size_t)N * N * N;
  double sumI = 0.0;
  for (int g = 0; g < a.copies; ++g) {
    unsigned long long* hb = a.heavy + ((size_t)slot * a.copies + g) * nw * T3;
    for (int cell = threadIdx.x; cell < T3; cell += kBlock) {
      const int lx = cell / (TS * TS), ly = (cell / TS) % TS, lz = cell % TS;
      const size_t lin = ((size_t)(o3[0] + lx) * N + (o3[1] + ly)) * N + (o3[2] + lz);
      put_node<T, false>(hb + cell, T3, a.ngrid, false, 0, inv_scale, out + (size_t)g * a.ngrid * N3 + lin, N3);
      if (wr >= 0 && g == 0) {
        const double v = a.scal->alpha * (double)(long long)hb[(size_t)wr * T3 + cell] * inv_scale;
        sumI += v * v * v;
      }
      // the slot starts the next measurement at zero (each word read by this thread only)
      for (int k = 0; k < nw; ++k) hb[(size_t)k * T3 + cell] = 0ull;
    }
  }
  if (wr >= 0) {
    sh[threadIdx.x] = sumI;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
      if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.tile_I[tile] = sh[0];
  }
}

// Work planning, one wavefront per tile: the tile's visits (its ranges summed
// across the lanes), its heavy slot, and for a split tile its parts after the
// first, appended to the extra work list. Work items are order-free (integer
// sums), so the append order does not matter.
__global__ void __launch_bounds__(kBlock) tile_parts_kernel(TileArgs a, int ntiles, int* hslot, int* heavy_tile,
                                                            int* nheavy, int* nextra, int2* extra) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (t >= ntiles) return;   // the whole wavefront leaves together
  int len = 0;
  if (lane < a.nr) {
    int st;
    tile_range(a, t, lane, &st, &len);
  }
  for (int off = 32; off > 0; off >>= 1) len += __shfl_xor(len, off);
  if (lane != 0) return;
  const int pv = part_visits(a.box_mode);
  const int np = (len + pv - 1) / pv;
  int hs = -1;
  if (np > 1) {
    const int sl = atomicAdd(nheavy, 1);
    if (sl < a.max_heavy) {   // out of slots: the tile runs whole
      hs = sl;
      heavy_tile[sl] = t;
      const int e = atomicAdd(nextra, np - 1);
      for (int q = 1; q < np; ++q) extra[e + q - 1] = make_int2(t, q);
    }
  }
  hslot[t] = hs;
}

// ----------------------------------------------------------------------------
// column assignment with the z transform (box-mode FP32 plans)
//
// A workgroup owns one column (kColW x kColW nodes in x and y, every z). The
// particles that reach it add their fixed-point contributions to the
// column's words in LDS, both grid copies at once, two channels per 64-bit
// word (as packed tiles do) at a scale of the column's own, from its visit
// count (order-free, so the result is bitwise reproducible). Every z line of
// the column is then transformed in LDS by the four-step scheme of the FFT
// passes (Sec. 2 sign convention) and only the kept frequencies |n_z| <= R_G
// are written, in the z pass's output layout: the assignment grids never
// reach device memory.

constexpr int kZBlock = 256;
constexpr int kColMaxRanges = 16;
constexpr int kZMaxGrids = 4;
constexpr int kZMaxLines = 2 * kZMaxGrids * kColW * kColW;

struct ZColArgs {
  int N, NC, p, copies, ngrid, RG, PG, nlines;
  int64_t PGs;                 // stored innermost extent of the output
  double wmax;                 // largest node weight of the kernel
  const int* start;            // bucket starts [NC^2 * 9 + 1]
  const DevScalars* scal;
  const float2* tw;            // e^{-2 pi i j / N}, j < N
  float2* out;                 // [copies * ngrid][N][N][PGs]
  // reads of one column: home column (cx - dx, cy - dy) and class range
  int nr;
  int rdx[kColMaxRanges], rdy[kColMaxRanges], rlo[kColMaxRanges], rhi[kColMaxRanges];
};

template <int N1, int N2>
__global__ void __launch_bounds__(kZBlock) zcol_kernel(ZColArgs a, Records<float> rec) {
  constexpr int N = N1 * N2;
  constexpr int LS = N2 * (N1 + 1) + 1;                     // LDS line stride (odd)
  static_assert(64 % N1 == 0, "a line's step-A tasks share a wavefront");
  extern __shared__ unsigned long long zacc[];              // [nlines][LS]
  __shared__ int r_st[kColMaxRanges], r_off[kColMaxRanges + 1];
  const int nb = a.NC * a.NC;
  int col = blockIdx.x;
  if (nb % 8 == 0) col = (col % 8) * (nb / 8) + col / 8;   // a band of neighbouring columns per XCD
  const int cx = col / a.NC, cy = col - cx * a.NC;
  const int x0 = cx * kColW, y0 = cy * kColW;
  int st = 0, en = 0;
  if (threadIdx.x < a.nr) {   // the column's bucket ranges, in flight while the words are cleared
    const int r = threadIdx.x;
    const int hx = (cx - a.rdx[r] + a.NC) % a.NC, hy = (cy - a.rdy[r] + a.NC) % a.NC;
    const int key = (hx * a.NC + hy) * kColClasses;
    st = a.start[key + a.rlo[r]];
    en = a.start[key + a.rhi[r]];
  }
  for (int i = threadIdx.x; i < a.nlines * LS / 2; i += kZBlock)   // nlines is a multiple of 4
    reinterpret_cast<ulonglong2*>(zacc)[i] = make_ulonglong2(0ull, 0ull);
  if (threadIdx.x < a.nr) {
    r_st[threadIdx.x] = st;
    r_off[threadIdx.x + 1] = en - st;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    r_off[0] = 0;
    for (int r = 0; r < a.nr; ++r) r_off[r + 1] += r_off[r];
  }
  __syncthreads();
  const int nv = r_off[a.nr];
  const int et = tile_exponent(nv, a.scal->cmax * a.wmax);
  const float tscale = ldexpf(1.0f, et);
  const int lg = kColW * kColW * LS;   // words between the lines of consecutive grids
  // visits range by range (the lanes of a wavefront mostly share a range, so
  // their stencils cross the column alike), each range in a scrambled order (a
  // multiplier prime to its length): neighbouring lanes take particles far
  // apart in the bucket order, which follows the catalogue's, so that their
  // atomics rarely share a word
  // a thread's next visit is loaded while the current one is added
  auto load_visit = [&](int v, double* u, float* c) {
    int r = 0;   // the range holding visit v: r_off[r] <= v < r_off[r + 1]
    for (int step = 8; step > 0; step >>= 1)
      if (r + step < a.nr && r_off[r + step] <= v) r += step;
    const int len = r_off[r + 1] - r_off[r];
    const int mult = len % 97 ? 97 : (len % 101 ? 101 : (len % 103 ? 103 : 1));
    const int64_t slot = (int64_t)r_st[r] + (int)(((int64_t)(v - r_off[r]) * mult) % len);
    const double* ru = rec.u(slot);
    u[0] = ru[0];
    u[1] = ru[1];
    u[2] = ru[2];
    const float* rc = rec.c(slot);
#pragma unroll
    for (int k = 0; k < 2 * kZMaxGrids; ++k) c[k] = k < 2 * a.ngrid ? rc[k] : 0.0f;
  };
  double nu[3] = {NAN, 0.0, 0.0};
  float nc[2 * kZMaxGrids];
  if (threadIdx.x < nv) load_visit(threadIdx.x, nu, nc);
#pragma unroll 1
  for (int v0 = threadIdx.x; v0 < nv; v0 += kZBlock) {
    const double u[3] = {nu[0], nu[1], nu[2]};
    float c[2 * kZMaxGrids];
#pragma unroll
    for (int k = 0; k < 2 * kZMaxGrids; ++k) c[k] = nc[k];
    if (v0 + kZBlock < nv) load_visit(v0 + kZBlock, nu, nc);
    if (!isfinite(u[0])) continue;
    for (int g = 0; g < a.copies; ++g) {
      int j[3];
      float w[3][3];
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) stencil_weights<float>(a.p, (float)stencil_param(u[ax] + 0.5 * g, a.p, &j[ax]), w[ax]);
      // the stencil nodes inside the column are consecutive: node j + s sits at
      // column-local index d + s, with d = j - (column start) taken periodically
      // into [-N/2, N/2); the loops run over those nodes only
      int dx = j[0] - x0, dy = j[1] - y0;
      dx += dx < -N / 2 ? N : (dx >= N / 2 ? -N : 0);
      dy += dy < -N / 2 ? N : (dy >= N / 2 ? -N : 0);
      const int sx1 = min(a.p, kColW - dx), sy0 = max(0, -dy), sy1 = min(a.p, kColW - dy);
      for (int sx = max(0, -dx); sx < sx1; ++sx) {
        const int lx = dx + sx;
        const float wxs = pick3(w[0], sx) * tscale;   // the column scale folded into the x weight
        for (int sy = sy0; sy < sy1; ++sy) {
          const int ly = dy + sy;
          const float wxy = wxs * pick3(w[1], sy);
          unsigned long long* line = zacc + (size_t)((g * a.ngrid * kColW + lx) * kColW + ly) * LS;
          for (int sz = 0; sz < a.p; ++sz) {
            int iz = j[2] + sz;
            iz += iz < 0 ? N : (iz >= N ? -N : 0);
            const float W = wxy * pick3(w[2], sz);
#pragma unroll
            for (int k = 0; k < kZMaxGrids; ++k) {
              if (k >= a.ngrid) break;
              atomicAdd(line + (size_t)k * lg + iz, pack2(__float2int_rn(c[2 * k] * W), __float2int_rn(c[2 * k + 1] * W)));
            }
          }
        }
      }
    }
  }
  __syncthreads();

  // step A: N2-point transforms of the strided subsequences of each line
  // (words converted on load), twiddled and written back transposed. The N1
  // tasks of a line are consecutive lanes of one wavefront (N1 divides 64),
  // whose reads of the line all precede its writes: no barrier inside.
  float2* lds = (float2*)zacc;
#pragma unroll 1
  for (int t = threadIdx.x; t < a.nlines * N1; t += kZBlock) {
    const int jl = t / N1, n1 = t - jl * N1;
    float2 vv[N2];
    const unsigned long long* wline = zacc + (size_t)jl * LS;
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
      int lo, hi;
      unpack2(wline[n1 + N1 * n2], &lo, &hi);
      vv[n2] = make_float2(ldexpf((float)lo, -et), ldexpf((float)hi, -et));
    }
    reg_fft<float, float2, N2>(vv, -1);
    float2* line = lds + (size_t)jl * LS;
#pragma unroll
    for (int i = 0; i < N2; ++i) {
      const int k2 = bit_reverse<N2>(i);
      const float2 tw = a.tw[(n1 * k2) % N];
      line[k2 * (N1 + 1) + n1] = make_float2(vv[i].x * tw.x - vv[i].y * tw.y, vv[i].x * tw.y + vv[i].y * tw.x);
    }
  }
  __syncthreads();

  // step C: N1-point transforms across n1; kept frequencies only
  for (int t = threadIdx.x; t < a.nlines * N2; t += kZBlock) {
    const int jl = t / N2, k2 = t - jl * N2;
    const float2* line = lds + (size_t)jl * LS + k2 * (N1 + 1);
    float2 uu[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) uu[n1] = line[n1];
    reg_fft<float, float2, N1>(uu, -1);
    const int ly = jl % kColW, lx = (jl / kColW) % kColW, b = jl / (kColW * kColW);   // b = copy * ngrid + grid
    float2* ob = a.out + ((int64_t)b * N + (x0 + lx)) * N * a.PGs + (int64_t)(y0 + ly) * a.PGs;
#pragma unroll
    for (int i = 0; i < N1; ++i) {
      int e = k2 + N2 * bit_reverse<N1>(i) + a.RG;   // stored entry of frequency k (n = e - R_G)
      if (e >= N) e -= N;
      if (e < a.PG) ob[e] = uu[i];
    }
  }
}

// y_L^M*(x^_node) on both grid copies in the complex-grid layout of the
// assignment output; transformed once per plan, it carries the box-mode mean
// subtraction into spectrum space.
struct YNodeArgs {
  double h, origin[3];
  int N, copies, ngrid;
  ChanInfo ci;
  int gre[kMaxGrids], gim[kMaxGrids];
  void* out;
};

template <typename T>
__global__ void __launch_bounds__(kBlock) ynode_fill_kernel(YNodeArgs a) {
  typedef typename cplx<T>::type T2;
  const int64_t N3 = (int64_t)a.N * a.N * a.N;
  const int64_t total = (int64_t)a.copies * N3;
  T2* out = (T2*)a.out;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
    const int g = (int)(i / N3);
    const int64_t lin = i - g * N3;
    const int ix = (int)(lin / ((int64_t)a.N * a.N)), iy = (int)((lin / a.N) % a.N), iz = (int)(lin % a.N);
    double u[3];
    node_dir(a.origin, a.h, a.ci.obs, ix, iy, iz, g, u);
    for (int gr = 0; gr < a.ngrid; ++gr) {
      T2 o;
      o.x = (T)node_y(a.ci, a.gre[gr], u[0], u[1], u[2]);
      o.y = a.gim[gr] >= 0 ? (T)node_y(a.ci, a.gim[gr], u[0], u[1], u[2]) : (T)0;
      out[((int64_t)g * a.ngrid + gr) * N3 + lin] = o;
    }
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

__global__ void zero_u64_kernel(unsigned long long* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

__global__ void zero_ints_kernel(int* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void zero_scal_kernel(DevScalars* s) {
  if (threadIdx.x == 0) {
    s->sum_w = s->sum_w_ran = s->sum_abs = s->sum_abs_ran = 0.0;
    s->alpha = s->scale = s->inv_scale = s->mean_cell = s->I = s->cmax = 0.0;
    s->err = 0;
    s->pad = 0;
  }
}

struct UnpackArgs {
  int gre[kMaxGrids], gim[kMaxGrids];
  int copies, ngrid, nch, N, box_mode;
  double h, origin[3];
  ChanInfo ci;
  const DevScalars* scal;
};

// Assignment grids in the [copy][channel][N^3] layout of the API, with the
// box-mode mean term (sum w / N^3) y_L^M*(x^_node) subtracted in FP64.
template <typename T>
__global__ void unpack_kernel(const void* grid, void* out, UnpackArgs m) {
  typedef typename cplx<T>::type T2;
  const T2* g = (const T2*)grid;
  T* o = (T*)out;
  const int64_t N3 = (int64_t)m.N * m.N * m.N;
  const int64_t total = (int64_t)m.copies * m.ngrid * N3;
  const double mean = m.scal->mean_cell;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cell = i % N3;
    const int64_t cg = i / N3;
    const int c = (int)(cg / m.ngrid), gr = (int)(cg % m.ngrid);
    const T2 v = g[i];
    double re = v.x, im = v.y;
    if (m.box_mode) {
      double u[3];
      node_dir(m.origin, m.h, m.ci.obs, (int)(cell / ((int64_t)m.N * m.N)), (int)((cell / m.N) % m.N),
               (int)(cell % m.N), c, u);
      re -= mean * node_y(m.ci, m.gre[gr], u[0], u[1], u[2]);
      if (m.gim[gr] >= 0) im -= mean * node_y(m.ci, m.gim[gr], u[0], u[1], u[2]);
    }
    o[((int64_t)c * m.nch + m.gre[gr]) * N3 + cell] = (T)re;
    if (m.gim[gr] >= 0) o[((int64_t)c * m.nch + m.gim[gr]) * N3 + cell] = (T)im;
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
  a.d = cat_ptrs(P, data);
  a.r = P.box_mode ? CatPtrs{} : cat_ptrs(P, rand);
  a.P0 = P.P0;
  a.inv_h = (double)P.N / P.L;
  for (int i = 0; i < 3; ++i) {
    a.origin[i] = P.origin[i];
    a.obs[i] = P.observer[i];
  }
  a.N = P.N;
  a.box_mode = P.box_mode;
  a.local = P.los_kind == TSB_LOS_LOCAL;
  DevScalars* scal = pass_scalars(P);
  a.scal = scal;
  a.partials = P.d_sum_partials;
  prof_begin(P, kStWeights, s);
  hipLaunchKernelGGL(zero_scal_kernel, dim3(1), dim3(64), 0, s, scal);
  hipLaunchKernelGGL(prep_kernel, dim3(kPrepBlocks), dim3(kBlock), 0, s, a);
  const double n3 = (double)P.N * P.N * P.N;
  hipLaunchKernelGGL(prep_final_kernel, dim3(1), dim3(kBlock), 0, s, (const double*)P.d_sum_partials,
                     kPrepBlocks, scal, P.box_mode, n3, P.L * P.L * P.L,
                     P.precision == TSB_FP64 ? 61 : 51, P.wpass ? (const DevScalars*)P.d_scal : nullptr);
  prof_end(P, kStWeights, s);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

// Record slots: two per complex grid, plus the randoms channel in survey mode.
static int record_slots(const Plan& P) { return 2 * (int)P.grids.size() + (P.box_mode ? 0 : 1); }

int record_stride(const Plan& P) {
  const int esz = P.precision == TSB_FP64 ? 8 : 4;
  return (24 + record_slots(P) * esz + 15) / 16 * 16;
}

// 64-bit fixed-point words per node held for one grid copy: one per record
// slot (packed FP32 tiles use the first ngrid of them).
int assign_words(const Plan& P) { return record_slots(P); }

int64_t assign_work_cap(const Plan& P, int64_t particles) {
  return work_capacity((int64_t)P.NT * P.NT * P.NT, particles, kPartVisits);
}

int assign_part_visits() { return kPartVisits; }   // the smaller of the two: more work items

int64_t assign_heavy_bytes(const Plan& P) {
  return (int64_t)P.heavy_slots * P.copies * assign_words(P) * P.T * P.T * P.T * 8;
}

// Slots for split tiles: a quarter of the tiles (dense catalogues split many),
// at least kMinHeavy, at most one per tile, and at most 1 GiB of sums or an
// eighth of the rest of the workspace (other_bytes), whichever is larger.
int assign_max_heavy(const Plan& P, int64_t other_bytes) {
  const int64_t ntiles = (int64_t)P.NT * P.NT * P.NT;
  const int64_t per = (int64_t)P.copies * assign_words(P) * P.T * P.T * P.T * 8;
  int64_t n = std::max<int64_t>(kMinHeavy, ntiles / 4);
  n = std::min<int64_t>(n, std::max<int64_t>(1LL << 30, other_bytes / 8) / per);
  n = std::max<int64_t>(n, kMinHeavy);
  return (int)std::min<int64_t>(n, ntiles);
}

int chan_info(const Plan& P, ChanInfo* ci) {
  *ci = ChanInfo{};
  ci->nch = (int)P.chans.size();
  if (ci->nch + 1 > kMaxCh || (int)P.grids.size() > kMaxGrids || record_slots(P) > kMaxCh)
    return fail(TSB_E_UNSUPPORTED, "too many channels");
  ci->local = P.los_kind == TSB_LOS_LOCAL;
  ci->window = P.estimator == TSB_WINDOW;
  for (int i = 0; i < 3; ++i) ci->obs[i] = P.observer[i];
  for (int c = 0; c < ci->nch; ++c) {
    ci->chL[c] = P.chans[c].L;
    ci->chM[c] = P.chans[c].M;
    ci->chPart[c] = P.chans[c].part;
  }
  ylm_norm_table(ci->ynorm);
  return TSB_OK;
}

// Reads of one tile, as (neighbour offset, class range): own tile every class;
// a neighbour at offset d only the classes whose stencils leave it towards the
// tile (class 2 on an axis with d = -1, class 0 with d = +1, any with d = 0).
// With NT = 2 the two neighbours of an axis coincide but take disjoint
// classes; with NT = 1 the own tile is the only read.
int tile_ranges(int NT, int* rd, int* rcl, int* rch) {
  int nr = 0;
  for (int dx = -1; dx <= 1; ++dx)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dz = -1; dz <= 1; ++dz) {
        if (NT == 1 && (dx || dy || dz)) continue;
        const int d = (dx + 1) * 9 + (dy + 1) * 3 + (dz + 1);
        auto opts = [](int dd, int* v) {
          if (dd < 0) { v[0] = 2; return 1; }
          if (dd > 0) { v[0] = 0; return 1; }
          v[0] = 0; v[1] = 1; v[2] = 2;
          return 3;
        };
        int vx[3], vy[3], vz[3];
        const int nx = opts(dx, vx), ny = opts(dy, vy), nz = opts(dz, vz);
        for (int i = 0; i < nx; ++i)
          for (int j = 0; j < ny; ++j)
            for (int k = 0; k < nz; ++k) {
              const int c = vx[i] * 9 + vy[j] * 3 + vz[k];
              if (nr > 0 && rd[nr - 1] == d && rch[nr - 1] == c) {
                rch[nr - 1] = c + 1;   // extends the previous range
              } else {
                rd[nr] = d;
                rcl[nr] = c;
                rch[nr] = c + 1;
                ++nr;
              }
            }
      }
  return nr;
}

template <typename T, int NCH>
int assign_front_impl(Plan& P, const BucketArgs& b, const ChanInfo& ci, hipStream_t s) {
  const int ntiles = P.NT * P.NT * P.NT;
  const int64_t ntot = b.d.n + b.r.n;
  const int nchx = ci.nch + (P.box_mode ? 0 : 1);
  const size_t lds = (size_t)assign_words(P) * P.T * P.T * P.T * sizeof(unsigned long long);
  // upper bound of the work items: a particle is visited by at most 8 tiles
  const int pv = part_visits(P.box_mode);
  const int64_t work_bound = (int64_t)ntiles + (8 * ntot + pv - 1) / pv + 1;
  if (work_bound > P.work_cap) return fail(TSB_E_UNSUPPORTED, "assignment: work list too small");
  if (P.tile_wgs <= 0) {
    // persistent workgroups of the tile kernel: as many as are resident at once
    int per_cu = 0, dev = 0, n_cu = 0;
    TSB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)assign_tile_kernel<T, NCH>,
                                                         kTileBlock, lds));
    TSB_HIP(hipGetDevice(&dev));
    TSB_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    P.tile_wgs = std::max(1, per_cu) * std::max(1, n_cu);
  }
  if (ntot > 0) {
    FillArgs<T, NCH> f;
    f.b = b;
    f.ci = ci;
    f.rec.cap = P.particle_cap;
    f.rec.base = (char*)P.d_rec;
    f.rec.stride = record_stride(P);
    f.nchx = nchx;
    f.zslot = -1;
    for (int gr = 0; gr < (int)P.grids.size(); ++gr) {
      f.slot_of[P.grids[gr].re] = 2 * gr;
      if (P.grids[gr].im >= 0)
        f.slot_of[P.grids[gr].im] = 2 * gr + 1;
      else
        f.zslot = 2 * gr + 1;
    }
    if (!P.box_mode) f.slot_of[ci.nch] = 2 * (int)P.grids.size();
    f.scal = pass_scalars(P);
    hipLaunchKernelGGL((bucket_fill_kernel<T, NCH>), dim3(grid_blocks(ntot)), dim3(kBlock), 0, s, f);
  }
  prof_end(P, kStBucket, s);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

// Everything after the bucketing: fixed launch shapes for a given plan and
// particle capacity (the work list lives in device memory), so the sequence
// can be captured into a graph.
template <typename T, int NCH>
int assign_back_impl(Plan& P, const ChanInfo& ci, hipStream_t s) {
  const int ntiles = P.NT * P.NT * P.NT;
  const int nw = assign_words(P);
  Records<T> rec;
  rec.cap = P.particle_cap;
  rec.base = (char*)P.d_rec;
  rec.stride = record_stride(P);
  TileArgs a{};
  a.inv_h = (double)P.N / P.L;
  a.h = P.L / (double)P.N;
  for (int i = 0; i < 3; ++i) a.origin[i] = P.origin[i];
  a.N = P.N;
  a.T = P.T;
  a.lt = P.T == 8 ? 3 : 2;
  a.NT = P.NT;
  a.p = P.p;
  a.copies = P.copies;
  a.box_mode = P.box_mode;
  a.ci = ci;
  a.ngrid = (int)P.grids.size();
  a.nw = nw;
  a.wr = P.box_mode ? -1 : nw - 1;
  a.wmax = P.p == 3 ? 0.421875 : 1.0;
  a.start = P.d_bk_start;
  a.scal = pass_scalars(P);
  a.out = P.d_grid;
  a.tile_I = P.d_sum_partials;
  a.nr = tile_ranges(P.NT, a.rd, a.rcl, a.rch);
  if (a.nr > kMaxRanges) return fail(TSB_E_UNSUPPORTED, "assignment: too many bucket ranges");
  int* nheavy = P.d_bk_count + P.nbk;   // heavy slots and extra parts: cleared with the bucket counts
  int* nextra = nheavy + 1;
  a.work = (const int2*)P.d_work;
  a.nextra = nextra;
  a.ntiles = ntiles;
  a.hslot = P.d_tile_hslot;
  a.heavy = (unsigned long long*)P.d_heavy;
  a.max_heavy = P.heavy_slots;
  prof_begin(P, kStAssign, s);
  // work items: tiles with more than part_visits visits are split into parts
  hipLaunchKernelGGL(tile_parts_kernel, dim3((ntiles + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0, s, a,
                     ntiles, P.d_tile_hslot, P.d_heavy_tile, nheavy, nextra, (int2*)P.d_work);
  const size_t lds = (size_t)nw * P.T * P.T * P.T * sizeof(unsigned long long);
  hipLaunchKernelGGL((assign_tile_kernel<T, NCH>), dim3(std::max(1, P.tile_wgs)), dim3(kTileBlock), lds, s, a,
                     rec);
  hipLaunchKernelGGL(heavy_final_kernel<T>, dim3(P.heavy_slots), dim3(kBlock), 0, s, a, (const int*)P.d_heavy_tile,
                     (const int*)nheavy);
  if (!P.box_mode) {
    const double vc = P.L * P.L * P.L / ((double)P.N * P.N * P.N);
    hipLaunchKernelGGL(norm_final_kernel, dim3(1), dim3(kBlock), 0, s, (const double*)P.d_sum_partials,
                       ntiles, pass_scalars(P), vc);
  }
  prof_end(P, kStAssign, s);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

// Reads of one column: home columns (cx - dx, cy - dy), dx, dy in 0..2, and
// the classes whose stencils reach at least dx columns up on x and dy on y,
// as contiguous class ranges (15 of them).
static int column_ranges(int* rdx, int* rdy, int* rlo, int* rhi) {
  int nr = 0;
  for (int dx = 0; dx <= 2; ++dx)
    for (int dy = 0; dy <= 2; ++dy)
      for (int rx = dx; rx <= 2; ++rx) {
        const int lo = rx * 3 + dy, hi = rx * 3 + 3;
        if (nr > 0 && rdx[nr - 1] == dx && rdy[nr - 1] == dy && rhi[nr - 1] == lo) {
          rhi[nr - 1] = hi;   // extends the previous range
          continue;
        }
        rdx[nr] = dx;
        rdy[nr] = dy;
        rlo[nr] = lo;
        rhi[nr] = hi;
        ++nr;
      }
  return nr;
}

static int zcol_lines(const Plan& P) { return P.copies * (int)P.grids.size() * kColW * kColW; }

static bool zcol_split(int N, int* n1, int* n2) {
  switch (N) {
    case 32: *n1 = 4; *n2 = 8; return true;
    case 64: *n1 = 8; *n2 = 8; return true;
    case 128: *n1 = 8; *n2 = 16; return true;
    case 256: *n1 = 16; *n2 = 16; return true;
    default: return false;
  }
}

int64_t zcol_lds_bytes(const Plan& P) {
  int n1 = 0, n2 = 0;
  if (!zcol_split(P.N, &n1, &n2)) return 0;
  return (int64_t)zcol_lines(P) * (n2 * (n1 + 1) + 1) * 8;
}

// Box-mode FP32 plans on a power-of-two grid of 32 to 256 points with at
// most four complex grids per copy.
bool zcol_applies(const Plan& P) {
  int n1 = 0, n2 = 0;
  if (P.precision != TSB_FP32 || !P.box_mode || !zcol_split(P.N, &n1, &n2)) return false;
  if ((int)P.grids.size() > kZMaxGrids || record_slots(P) != 2 * (int)P.grids.size()) return false;
  return zcol_lds_bytes(P) <= 96 * 1024;
}

// Bucket keys of the plan's assignment: the tiles' (tile, class) keys, or the
// columns' (column, class) keys if more.
int64_t assign_bucket_keys(const Plan& P) {
  const int64_t tiles = (int64_t)P.NT * P.NT * P.NT * kClasses;
  const int64_t NC = P.N / kColW;
  return P.zcol ? std::max(tiles, NC * NC * kColClasses) : tiles;
}

template <int N1, int N2>
static int launch_zcol(Plan& P, hipStream_t s) {
  ZColArgs a{};
  a.N = P.N;
  a.NC = P.N / kColW;
  a.p = P.p;
  a.copies = P.copies;
  a.ngrid = (int)P.grids.size();
  a.RG = P.RG;
  a.PG = P.PG;
  a.nlines = zcol_lines(P);
  a.PGs = pad_line(P.PG);
  a.wmax = P.p == 3 ? 0.421875 : 1.0;
  a.start = P.d_bk_start;
  a.scal = pass_scalars(P);
  a.tw = (const float2*)P.d_tw_n;
  a.out = (float2*)P.d_t1;
  a.nr = column_ranges(a.rdx, a.rdy, a.rlo, a.rhi);
  if (a.nr > kColMaxRanges || a.nlines > kZMaxLines) return fail(TSB_E_UNSUPPORTED, "column assignment: bad shape");
  Records<float> rec;
  rec.cap = P.particle_cap;
  rec.base = (char*)P.d_rec;
  rec.stride = record_stride(P);
  const size_t lds = (size_t)zcol_lds_bytes(P);
  prof_begin(P, kStAssign, s);
  hipLaunchKernelGGL((zcol_kernel<N1, N2>), dim3(a.NC * a.NC), dim3(kZBlock), lds, s, a, rec);
  prof_end(P, kStAssign, s);
  TSB_HIP(hipGetLastError());
  P.zcol_pass = 1;   // the forward transform starts at the y pass
  return TSB_OK;
}

static int run_zcol(Plan& P, hipStream_t s) {
  switch (P.N) {
    case 32: return launch_zcol<4, 8>(P, s);
    case 64: return launch_zcol<8, 8>(P, s);
    case 128: return launch_zcol<8, 16>(P, s);
    case 256: return launch_zcol<16, 16>(P, s);
    default: return fail(TSB_E_UNSUPPORTED, "column assignment: unsupported grid");
  }
}

int run_assign(Plan& P, const tsb_catalog* data, const tsb_catalog* rand, hipStream_t s) {
  BucketArgs b{};
  b.d = cat_ptrs(P, data);
  b.r = P.box_mode ? CatPtrs{} : cat_ptrs(P, rand);
  b.inv_h = (double)P.N / P.L;
  for (int i = 0; i < 3; ++i) b.origin[i] = P.origin[i];
  b.P0 = P.P0;
  b.N = P.N;
  b.T = P.T;
  b.NT = P.NT;
  b.p = P.p;
  b.copies = P.copies;
  b.box_mode = P.box_mode;
  b.count = P.d_bk_count;
  b.start = P.d_bk_start;
  b.keys = P.d_keys;
  b.colmode = zcol_active(P) ? 1 : 0;
  const int64_t ntot = b.d.n + b.r.n;
  const int64_t nbk = b.colmode ? (int64_t)(P.N / kColW) * (P.N / kColW) * kColClasses : P.nbk;
  const int nparts = (int)((nbk + kScanChunk - 1) / kScanChunk);
  prof_begin(P, kStBucket, s);
  // counts and the heavy-slot counters are adjacent: one fill clears them
  hipLaunchKernelGGL(zero_ints_kernel, dim3(grid_blocks(P.nbk + 2)), dim3(kBlock), 0, s, P.d_bk_count, P.nbk + 2);
  if (ntot > 0)
    hipLaunchKernelGGL(bucket_count_kernel, dim3(grid_blocks(ntot)), dim3(kBlock), 0, s, b);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(nparts), dim3(kBlock), 0, s, (const int*)P.d_bk_count, nbk,
                     P.d_scan_part);
  hipLaunchKernelGGL(scan_parts_kernel, dim3(1), dim3(kBlock), 0, s, P.d_scan_part, nparts);
  hipLaunchKernelGGL(scan_out_kernel, dim3(nparts), dim3(kBlock), 0, s, (const int*)P.d_bk_count, nbk,
                     (const int*)P.d_scan_part, P.d_bk_start);

  ChanInfo ci;
  if (int rc = chan_info(P, &ci)) return rc;
  const int nreg = record_slots(P);
  const bool f64 = P.precision == TSB_FP64;
  if (nreg <= 8) return f64 ? assign_front_impl<double, 8>(P, b, ci, s) : assign_front_impl<float, 8>(P, b, ci, s);
  if (nreg <= 16)
    return f64 ? assign_front_impl<double, 16>(P, b, ci, s) : assign_front_impl<float, 16>(P, b, ci, s);
  if (nreg <= 24)
    return f64 ? assign_front_impl<double, 24>(P, b, ci, s) : assign_front_impl<float, 24>(P, b, ci, s);
  return f64 ? assign_front_impl<double, kMaxCh>(P, b, ci, s) : assign_front_impl<float, kMaxCh>(P, b, ci, s);
}

int run_assign_back(Plan& P, hipStream_t s) {
  if (zcol_active(P)) return run_zcol(P, s);
  ChanInfo ci;
  if (int rc = chan_info(P, &ci)) return rc;
  const int nreg = record_slots(P);
  const bool f64 = P.precision == TSB_FP64;
  if (nreg <= 8) return f64 ? assign_back_impl<double, 8>(P, ci, s) : assign_back_impl<float, 8>(P, ci, s);
  if (nreg <= 16) return f64 ? assign_back_impl<double, 16>(P, ci, s) : assign_back_impl<float, 16>(P, ci, s);
  if (nreg <= 24) return f64 ? assign_back_impl<double, 24>(P, ci, s) : assign_back_impl<float, 24>(P, ci, s);
  return f64 ? assign_back_impl<double, kMaxCh>(P, ci, s) : assign_back_impl<float, kMaxCh>(P, ci, s);
}

int run_unpack_grids(Plan& P, void* out, hipStream_t s) {
  UnpackArgs m{};
  for (size_t g = 0; g < P.grids.size(); ++g) {
    m.gre[g] = P.grids[g].re;
    m.gim[g] = P.grids[g].im;
  }
  m.copies = P.copies;
  m.ngrid = (int)P.grids.size();
  m.nch = (int)P.chans.size();
  m.N = P.N;
  m.box_mode = P.box_mode;
  m.h = P.L / (double)P.N;
  for (int i = 0; i < 3; ++i) m.origin[i] = P.origin[i];
  if (int rc = chan_info(P, &m.ci)) return rc;
  m.scal = P.d_scal;
  const int64_t total = (int64_t)P.copies * (int64_t)P.grids.size() * P.N * P.N * P.N;
  if (P.precision == TSB_FP64)
    hipLaunchKernelGGL(unpack_kernel<double>, dim3(grid_blocks(total)), dim3(kBlock), 0, s, (const void*)P.d_grid,
                       out, m);
  else
    hipLaunchKernelGGL(unpack_kernel<float>, dim3(grid_blocks(total)), dim3(kBlock), 0, s, (const void*)P.d_grid,
                       out, m);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

// Sbar_L^M of the shot noise (Sec. 4.2, eq. 46): per real channel c (part of
// w y_L^M*), sum_gal w^3 ch_c(x^) - alpha^3 sum_ran w^3 ch_c(x^), as FP64 sums per
// block added in a fixed order.
template <int NCH>
struct SbarArgs {
  CatPtrs d, r;
  double P0;
  ChanInfo ci;
  const DevScalars* scal;
  double* partials;   // [gridDim][nch]
};

template <int NCH>
__global__ void __launch_bounds__(kBlock) sbar_kernel(SbarArgs<NCH> a) {
  __shared__ double sh[kBlock];
  const double alpha = a.scal->alpha;
  double acc[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) acc[c] = 0.0;
  const int64_t ntot = a.d.n + a.r.n;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < ntot; i += (int64_t)gridDim.x * kBlock) {
    const bool ran = i >= a.d.n;
    const CatPtrs& c = ran ? a.r : a.d;
    const int64_t j = ran ? i - a.d.n : i;
    const double w = particle_weight(c, j, a.P0);
    if (!isfinite(w) || !isfinite((double)c.x[j]) || !isfinite((double)c.y[j]) || !isfinite((double)c.z[j]))
      continue;   // reported by the weight pass
    double cv[NCH];
    // w^3 and alpha^3: galaxies w^3 y*, randoms -alpha^3 w^3 y*
    channel_values<NCH>(a.ci, c.x[j], c.y[j], c.z[j], w * w * w, ran, alpha * alpha * alpha, cv);
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) acc[ch] += ch < a.ci.nch ? cv[ch] : 0.0;
  }
  for (int ch = 0; ch < a.ci.nch; ++ch) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < NCH; ++k) v = k == ch ? acc[k] : v;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
      if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.partials[(size_t)blockIdx.x * a.ci.nch + ch] = sh[0];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kBlock) sbar_final_kernel(const double* partials, int nblocks, int nch,
                                                            double* out) {
  __shared__ double sh[kBlock];
  for (int ch = 0; ch < nch; ++ch) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kBlock) v += partials[(size_t)b * nch + ch];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
      if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[ch] = sh[0];
    __syncthreads();
  }
}

template <int NCH>
int sbar_impl(Plan& P, const tsb_catalog* data, const tsb_catalog* rand, hipStream_t s) {
  SbarArgs<NCH> a{};
  const int saved = P.wpass;
  P.wpass = 0;
  a.d = cat_ptrs(P, data);
  a.r = P.box_mode ? CatPtrs{} : cat_ptrs(P, rand);
  P.wpass = saved;
  a.P0 = P.P0;
  if (int rc = chan_info(P, &a.ci)) return rc;
  a.scal = P.d_scal;
  a.partials = P.d_sum_partials;   // (free between the weight pass and the tiles)
  hipLaunchKernelGGL((sbar_kernel<NCH>), dim3(kPrepBlocks), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(sbar_final_kernel, dim3(1), dim3(kBlock), 0, s, (const double*)P.d_sum_partials, kPrepBlocks,
                     a.ci.nch, P.d_sbar);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

// Clear `bytes` (a multiple of 8) of device memory with a kernel (no memset
// node: the call may be captured into a graph).
int run_fill_zero(void* p, int64_t bytes, hipStream_t s) {
  const int64_t n = bytes / 8;
  if (n <= 0) return TSB_OK;
  hipLaunchKernelGGL(zero_u64_kernel, dim3(grid_blocks(n)), dim3(kBlock), 0, s, (unsigned long long*)p, n);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

int run_sbar(Plan& P, const tsb_catalog* data, const tsb_catalog* rand, hipStream_t s) {
  const int nch = (int)P.chans.size();
  if (nch <= 8) return sbar_impl<8>(P, data, rand, s);
  if (nch <= 16) return sbar_impl<16>(P, data, rand, s);
  if (nch <= 24) return sbar_impl<24>(P, data, rand, s);
  return sbar_impl<kMaxCh>(P, data, rand, s);
}

int run_ynode_fill(Plan& P, hipStream_t s) {
  YNodeArgs y{};
  y.h = P.L / (double)P.N;
  for (int i = 0; i < 3; ++i) y.origin[i] = P.origin[i];
  y.N = P.N;
  y.copies = P.copies;
  y.ngrid = (int)P.grids.size();
  if (int rc = chan_info(P, &y.ci)) return rc;
  for (int g = 0; g < y.ngrid; ++g) {
    y.gre[g] = P.grids[g].re;
    y.gim[g] = P.grids[g].im;
  }
  y.out = P.d_grid;
  const int64_t total = (int64_t)P.copies * P.N * P.N * P.N;
  if (P.precision == TSB_FP64)
    hipLaunchKernelGGL(ynode_fill_kernel<double>, dim3(grid_blocks(total)), dim3(kBlock), 0, s, y);
  else
    hipLaunchKernelGGL(ynode_fill_kernel<float>, dim3(grid_blocks(total)), dim3(kBlock), 0, s, y);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

}  // namespace tsb
