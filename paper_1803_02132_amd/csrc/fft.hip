// Batched 3D FFTs as three 1D passes, each a workgroup-per-line-block kernel:
// a block of lines is loaded into LDS with coalesced reads (consecutive lines
// are adjacent in memory for the strided axes), transformed by an in-LDS
// Stockham autosort FFT (radix 4, 2 and 3), and written back. Passes read and
// write only the stored ("pruned") part of each axis: the forward transform
// keeps frequencies |n_i| <= R, the inverse starts from them.
//
// Forward (Sec. 2 sign convention e^{-ik.x}): grids -> spectra cube, then the
// interlace combination and W_mass deconvolution (Sec. 4.2, eq. 39).
// Inverse (eq. 42): F_l^m(x; k) from the shell-filtered spectrum, G_L^M(x)
// from the band-limited spectrum, on the reduction grid M.
#include <cmath>

#include "tsb_internal.h"
#include "fft_reg.h"

namespace tsb {

namespace {

constexpr int kMaxParts = 2;

template <typename T>
struct PassArgs {
  typedef typename cplx<T>::type T2;
  const T2* in;
  T2* out;
  const T2* tw;            // e^{-2 pi i k / N}, k < N
  int64_t in_bs, out_bs;   // batch strides (elements)
  int64_t in_sa, in_sb, in_se, out_sa, out_sb, out_se;
  int nbatch, dA, dB;      // lines indexed (batch, a, b)
  int in_cnt, out_cnt;     // stored entries along the axis
  int in_off, out_off;     // stored entry e <-> frequency / position e - off (mod N)
  int N, dir;              // FFT length; -1 forward, +1 inverse
  int lpw;                 // lines per workgroup (consecutive b)
  int contiguous;          // element stride 1 (else b stride 1)
  // pre-operation on loaded values
  int pre;                 // 0 none, 1 band mask |n|^2 <= n2max, 2 shell filter,
                           // 3 times the slot's separation kernel (3PCF),
                           // 4 shell filter of each part's own source spectrum
  int offA, offB, offE;    // frequency = index - off for a, b, e
  int axA, axB, axE;       // which Cartesian axis (0 x, 1 y, 2 z) a, b and e index
  int64_t n2max;
  const int* bin_lut;      // shell of n^2 (n^2 <= lut_max), -1 none
  int64_t lut_max;
  const FKind* kinds;
  int nkinds;
  const void* kslot;       // pre 3: [batch][in cube layout] separation kernels
  int64_t kslot_bs;
  const void* spec;        // pre 4: spectra [grid][PG^3], frequency n at n + RG per axis
  int RG;
  // Sparsity of shell-filtered or band-limited spectra: a line, or an entry,
  // whose frequency coordinates alone give |n|^2 above r2 holds zeros; such a
  // line is neither read nor written, such an entry not read (every consumer
  // of the pass buffers applies the same rule). r2 = sp_r2[batch / sp_div], or
  // sp_c when sp_r2 is null; sp_a, sp_b, sp_e: the offset that turns index a,
  // b, e into a frequency (-1: the index is a position and does not count).
  int sp;
  const int* sp_r2;
  int sp_div;
  int64_t sp_c;
  int sp_a, sp_b, sp_e;
  // Output-side band limit of the forward passes: an output entry e of line
  // (a, b) whose frequencies (a - so_a, b - so_b, e - so_e; -1: not counted)
  // give |n|^2 above so_r2 is never read (the inverse chains and the
  // combination stop at the band limit) and is not written (so_on = 0: off).
  int so_on;
  int64_t so_r2;
  int so_a, so_b, so_e;
  // forward x pass with the combination (fft4_combine_kernel): copies of each
  // grid, the input stride between them, the per-axis table of combine_kernel,
  // the box-mode mean term (or null), the scalars holding its mean, DC zeroing
  int cb_copies;
  int64_t cb_copy_bs;
  const double* cb_tab;
  const T2* cb_yspec;
  const DevScalars* cb_scal;
  int cb_box;
  double ynorm[45];
};

// Live lines [*lo, *hi) of a workgroup's lines [b0, b0 + nl) under the
// sparsity rule, and the squared frequency of index a (false: none live).
template <typename T>
__device__ inline bool sparse_lines(const PassArgs<T>& a, int batch, int ia, int b0, int nl, int64_t* r2,
                                    int64_t* fa2, int* lo, int* hi) {
  *lo = b0;
  *hi = b0 + nl;
  *fa2 = 0;
  *r2 = 0;
  if (!a.sp) return true;
  *r2 = a.sp_r2 ? (int64_t)a.sp_r2[batch / a.sp_div] : a.sp_c;
  if (a.sp_a >= 0) *fa2 = (int64_t)(ia - a.sp_a) * (ia - a.sp_a);
  const int64_t rem = *r2 - *fa2;
  if (rem < 0) return false;
  if (a.sp_b >= 0) {
    int h = (int)sqrt((double)rem);
    while ((int64_t)h * h > rem) --h;
    while ((int64_t)(h + 1) * (h + 1) <= rem) ++h;
    *lo = max(*lo, a.sp_b - h);
    *hi = min(*hi, a.sp_b + h + 1);
  }
  return *lo < *hi;
}

// Whether output entry e of line (ia, b) lies beyond the output band limit.
template <typename T>
__device__ inline bool beyond_out(const PassArgs<T>& a, int ia, int b, int e) {
  if (!a.so_on) return false;
  int64_t f = 0;
  if (a.so_a >= 0) f += (int64_t)(ia - a.so_a) * (ia - a.so_a);
  if (a.so_b >= 0) f += (int64_t)(b - a.so_b) * (b - a.so_b);
  if (a.so_e >= 0) f += (int64_t)(e - a.so_e) * (e - a.so_e);
  return f > a.so_r2;
}

// Whether stored entry e of line b is a zero of the sparsity rule.
template <typename T>
__device__ inline bool sparse_zero(const PassArgs<T>& a, int64_t r2, int64_t fa2, int b, int e) {
  if (!a.sp) return false;
  int64_t f = fa2;
  if (a.sp_b >= 0) f += (int64_t)(b - a.sp_b) * (b - a.sp_b);
  if (a.sp_e >= 0) f += (int64_t)(e - a.sp_e) * (e - a.sp_e);
  return f > r2;
}

template <typename T2, typename T>
__device__ inline T2 cmul(T2 a, T2 b) {
  T2 r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

template <typename T>
__device__ inline typename cplx<T>::type shell_value(const PassArgs<T>& a, int batch, int fa, int fb,
                                                     int fe, typename cplx<T>::type v) {
  // F slot input (eq. 42 with eq. 38): sum_parts factor * y_l^m*(k^) * dn(k) on shell b
  typedef typename cplx<T>::type T2;
  T2 zero;
  zero.x = 0;
  zero.y = 0;
  const int64_t n2 = (int64_t)fa * fa + (int64_t)fb * fb + (int64_t)fe * fe;
  if (n2 == 0 || n2 > a.lut_max) return zero;
  const int bin = a.bin_lut[n2];
  if (bin != batch / a.nkinds) return zero;
  const FKind& k = a.kinds[batch % a.nkinds];   // read in place (no private copy)
  const double r = sqrt((double)n2);
  // unit vector: a, b, e index the Cartesian axes axA, axB, axE
  const double ca = fa / r, cb = fb / r, ce = fe / r;
  const double ux = a.axA == 0 ? ca : (a.axB == 0 ? cb : ce);
  const double uy = a.axA == 1 ? ca : (a.axB == 1 ? cb : ce);
  const double uz = a.axA == 2 ? ca : (a.axB == 2 ? cb : ce);
  double fr = 0.0, fi = 0.0;
  for (int p = 0; p < k.nparts; ++p) {
    double yr, yi;
    ylm_pos_m(k.part[p].l, k.part[p].m, ux, uy, uz, a.ynorm, &yr, &yi);
    // factor * conj(y)
    fr += k.part[p].fr * yr + k.part[p].fi * yi;
    fi += k.part[p].fi * yr - k.part[p].fr * yi;
  }
  T2 o;
  o.x = (T)(fr * (double)v.x - fi * (double)v.y);
  o.y = (T)(fr * (double)v.y + fi * (double)v.x);
  return o;
}

template <typename T>
__device__ inline typename cplx<T>::type shell_value_src(const PassArgs<T>& a, int batch, int fa, int fb,
                                                         int fe, typename cplx<T>::type v) {
  // F slot input of the first-vertex LOS: sum_parts factor * y_l^m*(k^) * S_part(k)
  // on shell b, S_part = dn_0^0 (the loaded value) or dn_L^M from a grid spectrum
  typedef typename cplx<T>::type T2;
  T2 zero;
  zero.x = 0;
  zero.y = 0;
  const int64_t n2 = (int64_t)fa * fa + (int64_t)fb * fb + (int64_t)fe * fe;
  if (n2 == 0 || n2 > a.lut_max) return zero;
  const int bin = a.bin_lut[n2];
  if (bin != batch / a.nkinds) return zero;
  const FKind& k = a.kinds[batch % a.nkinds];
  const double r = sqrt((double)n2);
  const double ca = fa / r, cb = fb / r, ce = fe / r;
  const double ux = a.axA == 0 ? ca : (a.axB == 0 ? cb : ce);
  const double uy = a.axA == 1 ? ca : (a.axB == 1 ? cb : ce);
  const double uz = a.axA == 2 ? ca : (a.axB == 2 ? cb : ce);
  const int nx = a.axA == 0 ? fa : (a.axB == 0 ? fb : fe);
  const int ny = a.axA == 1 ? fa : (a.axB == 1 ? fb : fe);
  const int nz = a.axA == 2 ? fa : (a.axB == 2 ? fb : fe);
  const int PG = 2 * a.RG + 1;
  const int64_t pg3 = (int64_t)PG * PG * PG;
  const int64_t ip = ((int64_t)(nx + a.RG) * PG + (ny + a.RG)) * PG + (nz + a.RG);
  const int64_t im = ((int64_t)(a.RG - nx) * PG + (a.RG - ny)) * PG + (a.RG - nz);
  double fr = 0.0, fi = 0.0;
  for (int p = 0; p < k.nparts; ++p) {
    const FPart& fp = k.part[p];
    const int am = fp.m < 0 ? -fp.m : fp.m;
    double yr, yi;
    ylm_pos_m(fp.l, am, ux, uy, uz, a.ynorm, &yr, &yi);
    if (fp.m < 0) {   // y_l^-m = (-1)^m conj(y_l^m)
      const double sg = (am & 1) ? -1.0 : 1.0;
      yr *= sg;
      yi *= -sg;
    }
    double sr = (double)v.x, si = (double)v.y;
    if (fp.src >= 0) {
      const T2* S = (const T2*)a.spec + (int64_t)fp.src * pg3;
      const T2 s0 = S[ip];
      sr = (double)s0.x;
      si = (double)s0.y;
      if (fp.smode != 0) {
        const T2 s1 = S[im];
        if (fp.smode == 1) {   // (S(k) + conj S(-k)) / 2
          sr = 0.5 * ((double)s0.x + (double)s1.x);
          si = 0.5 * ((double)s0.y - (double)s1.y);
        } else {               // (S(k) - conj S(-k)) / (2i)
          sr = 0.5 * ((double)s0.y + (double)s1.y);
          si = -0.5 * ((double)s0.x - (double)s1.x);
        }
      }
    }
    // factor * conj(y) * S
    const double cr = fp.fr * yr + fp.fi * yi, ci = fp.fi * yr - fp.fr * yi;
    fr += cr * sr - ci * si;
    fi += cr * si + ci * sr;
  }
  T2 o;
  o.x = (T)fr;
  o.y = (T)fi;
  return o;
}

template <typename T>
__device__ inline typename cplx<T>::type apply_pre(const PassArgs<T>& a, int batch, int ia, int ib, int e,
                                                   typename cplx<T>::type v) {
  typedef typename cplx<T>::type T2;
  const int fa = ia - a.offA, fb = ib - a.offB, fe = e - a.offE;
  if (a.pre == 4) return shell_value_src<T>(a, batch, fa, fb, fe, v);
  if (a.pre == 3) {
    const T2 k = ((const T2*)a.kslot)[(int64_t)batch * a.kslot_bs + (int64_t)ia * a.in_sa +
                                      (int64_t)ib * a.in_sb + (int64_t)e * a.in_se];
    return cmul<T2, T>(v, k);
  }
  if (a.pre == 1) {
    const int64_t n2 = (int64_t)fa * fa + (int64_t)fb * fb + (int64_t)fe * fe;
    if (n2 > a.n2max) {
      T2 z;
      z.x = 0;
      z.y = 0;
      return z;
    }
    return v;
  }
  return shell_value<T>(a, batch, fa, fb, fe, v);
}


template <typename T>
__global__ void __launch_bounds__(kBlock) fft_pass_kernel(PassArgs<T> a) {
  typedef typename cplx<T>::type T2;
  extern __shared__ char smem[];
  const int N = a.N, NP = a.N + 1;
  T2* buf0 = (T2*)smem;
  T2* buf1 = buf0 + (size_t)a.lpw * NP;
  const int nbb = (a.dB + a.lpw - 1) / a.lpw;
  const int64_t blk = blockIdx.x;
  const int bb = (int)(blk % nbb);
  const int64_t rest = blk / nbb;
  const int ia = (int)(rest % a.dA);
  const int batch = (int)(rest / a.dA);
  int b0 = bb * a.lpw;
  int nl = min(a.lpw, a.dB - b0);
  const int tid = threadIdx.x;
  int64_t r2, fa2;
  int blo, bhi;
  if (!sparse_lines(a, batch, ia, b0, nl, &r2, &fa2, &blo, &bhi)) return;   // uniform: no live line
  b0 = blo;
  nl = bhi - blo;

  T2 zero;
  zero.x = 0;
  zero.y = 0;
  if (a.in_cnt < N)
    for (int i = tid; i < nl * NP; i += kBlock) buf0[i] = zero;
  __syncthreads();

  // ---- load ------------------------------------------------------------------
  const T2* inb = a.in + (int64_t)batch * a.in_bs + (int64_t)ia * a.in_sa;
  for (int idx = tid; idx < nl * a.in_cnt; idx += kBlock) {
    int j, e;
    if (a.contiguous) {
      j = idx / a.in_cnt;
      e = idx - j * a.in_cnt;
    } else {
      e = idx / nl;
      j = idx - e * nl;
    }
    T2 v = zero;
    if (!sparse_zero(a, r2, fa2, b0 + j, e)) {
      v = inb[(int64_t)(b0 + j) * a.in_sb + (int64_t)e * a.in_se];
      if (a.pre) v = apply_pre<T>(a, batch, ia, b0 + j, e, v);
    }
    int pos = e - a.in_off;
    if (pos < 0) pos += N;
    buf0[j * NP + pos] = v;
  }
  __syncthreads();

  // ---- Stockham stages ----------------------------------------------------------
  T2* src = buf0;
  T2* dst = buf1;
  int Ns = 1, rem = N;
  const T sgn = (T)a.dir;
  while (Ns < N) {
    const int r = (rem % 4 == 0) ? 4 : ((rem % 2 == 0) ? 2 : 3);
    const int nbf = N / r;
    const int tstride = N / (Ns * r);
    for (int idx = tid; idx < nl * nbf; idx += kBlock) {
      const int line = idx / nbf;
      const int jj = idx - line * nbf;
      const T2* s = src + line * NP;
      T2* d = dst + line * NP;
      const int k = jj % Ns;
      T2 v[4];
      for (int t = 0; t < r; ++t) v[t] = s[jj + t * nbf];
      if (k) {
        for (int t = 1; t < r; ++t) {
          T2 w = a.tw[t * k * tstride];
          if (a.dir > 0) w.y = -w.y;   // tw holds e^{-i...}; the inverse uses its conjugate
          v[t] = cmul<T2, T>(v[t], w);
        }
      }
      if (r == 4) {
        T2 t0, t1, t2, t3;
        t0.x = v[0].x + v[2].x; t0.y = v[0].y + v[2].y;
        t1.x = v[0].x - v[2].x; t1.y = v[0].y - v[2].y;
        t2.x = v[1].x + v[3].x; t2.y = v[1].y + v[3].y;
        // (v1 - v3) * (sgn i)
        const T dx = v[1].x - v[3].x, dy = v[1].y - v[3].y;
        t3.x = -sgn * dy;
        t3.y = sgn * dx;
        v[0].x = t0.x + t2.x; v[0].y = t0.y + t2.y;
        v[2].x = t0.x - t2.x; v[2].y = t0.y - t2.y;
        v[1].x = t1.x + t3.x; v[1].y = t1.y + t3.y;
        v[3].x = t1.x - t3.x; v[3].y = t1.y - t3.y;
      } else if (r == 2) {
        const T2 t0 = v[0];
        v[0].x = t0.x + v[1].x; v[0].y = t0.y + v[1].y;
        v[1].x = t0.x - v[1].x; v[1].y = t0.y - v[1].y;
      } else {
        const T c = (T)0.86602540378443864676;   // sqrt(3)/2
        T2 sm, df;
        sm.x = v[1].x + v[2].x; sm.y = v[1].y + v[2].y;
        df.x = v[1].x - v[2].x; df.y = v[1].y - v[2].y;
        T2 m;
        m.x = v[0].x - (T)0.5 * sm.x;
        m.y = v[0].y - (T)0.5 * sm.y;
        // sgn i c (v1 - v2)
        const T ux = -sgn * c * df.y, uy = sgn * c * df.x;
        v[0].x = v[0].x + sm.x; v[0].y = v[0].y + sm.y;
        v[1].x = m.x + ux; v[1].y = m.y + uy;
        v[2].x = m.x - ux; v[2].y = m.y - uy;
      }
      const int ob = (jj / Ns) * Ns * r + k;
      for (int t = 0; t < r; ++t) d[ob + t * Ns] = v[t];
    }
    __syncthreads();
    T2* tmp = src;
    src = dst;
    dst = tmp;
    Ns *= r;
    rem /= r;
  }

  // ---- store -------------------------------------------------------------------
  T2* outb = a.out + (int64_t)batch * a.out_bs + (int64_t)ia * a.out_sa;
  for (int idx = tid; idx < nl * a.out_cnt; idx += kBlock) {
    int j, e;
    if (a.contiguous) {
      j = idx / a.out_cnt;
      e = idx - j * a.out_cnt;
    } else {
      e = idx / nl;
      j = idx - e * nl;
    }
    int pos = e - a.out_off;
    if (pos < 0) pos += N;
    if (!beyond_out(a, ia, b0 + j, e)) outb[(int64_t)(b0 + j) * a.out_sb + (int64_t)e * a.out_se] = src[j * NP + pos];
  }
}

// Interlace combination and W_mass deconvolution on the stored cube
// (Sec. 4.2, eq. 39): S = (D1 + e^{i pi (nx+ny+nz)/N} D2)/2 / prod sinc(pi n_i/N)^p;
// in box mode the DC mode of dn_0^0 (real part of grid 0) is zero, and the
// mean term (sum w / N^3) y_L^M*(x^_node) of the local-LOS channels is removed
// here through its precomputed transform (it is linear in the grid).
template <typename T>
__global__ void __launch_bounds__(kBlock) combine_kernel(const typename cplx<T>::type* t3,
                                                         typename cplx<T>::type* spec, int ngrid,
                                                         int copies, int R, int box_mode,
                                                         const double* axis_tab,
                                                         const typename cplx<T>::type* yspec,
                                                         const DevScalars* scal) {
  // axis_tab: [P] 1/W_axis(n), then [P] cos(pi n/N), then [P] sin(pi n/N), n = index - R;
  // W and the interlace phase factor over the three axes. One row (grid, x, y)
  // per half workgroup, z across its lanes; the row's x and y factors are
  // formed once per row.
  typedef typename cplx<T>::type T2;
  const int P = 2 * R + 1;
  const double* iw = axis_tab;
  const double* pc = axis_tab + P;
  const double* ps = axis_tab + 2 * P;
  const int64_t P3 = (int64_t)P * P * P;
  const int rows = ngrid * P * P;
  const double mean = yspec ? scal->mean_cell : 0.0;
  for (int row = blockIdx.x * (kBlock / 128) + (threadIdx.x >> 7); row < rows; row += gridDim.x * (kBlock / 128))
  for (int iz = threadIdx.x & 127; iz < P; iz += 128) {
    const int g = row / (P * P), rxy = row - g * P * P, ix = rxy / P, iy = rxy - ix * P;
    const double czz = pc[iz], szz = ps[iz], wz = iw[iz];
    const int64_t i = (int64_t)row * P + iz;
    const T2 v1 = t3[i];
    double re = v1.x, im = v1.y;
    if (copies == 2) {
      const T2 v2 = t3[(int64_t)ngrid * P3 + i];
      // e^{i pi (nx+ny+nz)/N} as the product of the three axis phases
      const double cxy = pc[ix] * pc[iy] - ps[ix] * ps[iy], sxy = pc[ix] * ps[iy] + ps[ix] * pc[iy];
      const double c = cxy * czz - sxy * szz, sn = cxy * szz + sxy * czz;
      re = 0.5 * (re + c * (double)v2.x - sn * (double)v2.y);
      im = 0.5 * (im + c * (double)v2.y + sn * (double)v2.x);
    }
    const double inv_w = iw[ix] * iw[iy] * wz;
    re *= inv_w;
    im *= inv_w;
    if (yspec) {
      // box mode: minus (sum w / N^3) times the same transform of y_L^M*(x^_node)
      const T2 y = yspec[i];
      re -= mean * (double)y.x;
      im -= mean * (double)y.y;
    }
    if (box_mode && g == 0 && ix == R && iy == R && iz == R) re = 0.0;
    T2 o;
    o.x = (T)re;
    o.y = (T)im;
    spec[i] = o;
  }
}

// dn_0^0 on the F cube from the (0,0)-carrying grid 0: (S0(n) + conj(S0(-n)))/2.
template <typename T>
__global__ void __launch_bounds__(kBlock) dcube_kernel(const typename cplx<T>::type* spec0,
                                                       typename cplx<T>::type* dc, int RG, int RF) {
  typedef typename cplx<T>::type T2;
  const int PG = 2 * RG + 1, PF = 2 * RF + 1;
  const int64_t total = (int64_t)PF * PF * PF;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
    const int nx = (int)(i / ((int64_t)PF * PF)) - RF, ny = (int)((i / PF) % PF) - RF, nz = (int)(i % PF) - RF;
    const int64_t ip = ((int64_t)(nx + RG) * PG + (ny + RG)) * PG + (nz + RG);
    const int64_t im = ((int64_t)(-nx + RG) * PG + (-ny + RG)) * PG + (-nz + RG);
    const T2 a = spec0[ip], b = spec0[im];
    T2 o;
    o.x = (T)0.5 * (a.x + b.x);
    o.y = (T)0.5 * (a.y - b.y);
    dc[i] = o;
  }
}


// Four-step transform of lines of length N = N1 N2 (Sec. 2 sign convention):
// x[n1 + N1 n2] -> N2-point DFTs over n2 (per n1, in registers) -> twiddle
// W_N^{n1 k2} -> one LDS transpose -> N1-point DFTs over n1 (per k2) ->
// X[k2 + N2 k1]. Lines in a workgroup are consecutive in b; loads and stores
// walk the memory-contiguous index fastest.
template <typename T, int N1, int N2>
__global__ void __launch_bounds__(kBlock) fft4_kernel(PassArgs<T> a) {
  typedef typename cplx<T>::type T2;
  constexpr int N = N1 * N2;
  constexpr int LS = N2 * (N1 + 1) + 1;   // LDS line stride (odd: lines start in different banks)
  extern __shared__ char smem[];
  T2* lds = (T2*)smem;
  const int nbb = (a.dB + a.lpw - 1) / a.lpw;
  const int64_t blk = blockIdx.x;
  const int bb = (int)(blk % nbb);
  const int64_t rest = blk / nbb;
  const int ia = (int)(rest % a.dA);
  const int batch = (int)(rest / a.dA);
  int b0 = bb * a.lpw;
  int nl = min(a.lpw, a.dB - b0);
  int64_t r2, fa2;
  int blo, bhi;
  if (!sparse_lines(a, batch, ia, b0, nl, &r2, &fa2, &blo, &bhi)) return;   // uniform: no live line
  b0 = blo;
  nl = bhi - blo;
  const T2* inb = a.in + (int64_t)batch * a.in_bs + (int64_t)ia * a.in_sa;
  T2* outb = a.out + (int64_t)batch * a.out_bs + (int64_t)ia * a.out_sa;

  // ---- step A: N2-point transforms of the strided subsequences ---------------
  for (int task = threadIdx.x; task < nl * N1; task += kBlock) {
    int j, n1;
    if (a.contiguous) {
      j = task / N1;
      n1 = task - j * N1;
    } else {
      n1 = task / nl;
      j = task - n1 * nl;
    }
    T2 v[N2];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
      const int pos = n1 + N1 * n2;        // position in the line
      int e = pos + a.in_off;               // stored entry holding it
      if (e >= N) e -= N;
      T2 x;
      x.x = 0;
      x.y = 0;
      if (e < a.in_cnt && !sparse_zero(a, r2, fa2, b0 + j, e)) {
        x = inb[(int64_t)(b0 + j) * a.in_sb + (int64_t)e * a.in_se];
        if (a.pre) x = apply_pre<T>(a, batch, ia, b0 + j, e, x);
      }
      v[n2] = x;
    }
    reg_fft<T, T2, N2>(v, a.dir);
    T2* line = lds + j * LS;
#pragma unroll
    for (int i = 0; i < N2; ++i) {
      const int k2 = bit_reverse<N2>(i);
      T2 w = a.tw[(n1 * k2) % N];
      if (a.dir > 0) w.y = -w.y;
      T2 o;
      o.x = v[i].x * w.x - v[i].y * w.y;
      o.y = v[i].x * w.y + v[i].y * w.x;
      line[k2 * (N1 + 1) + n1] = o;
    }
  }
  __syncthreads();

  // ---- step C: N1-point transforms across n1 -----------------------------------
  for (int task = threadIdx.x; task < nl * N2; task += kBlock) {
    int j, k2;
    if (a.contiguous) {
      j = task / N2;
      k2 = task - j * N2;
    } else {
      k2 = task / nl;
      j = task - k2 * nl;
    }
    const T2* line = lds + j * LS + k2 * (N1 + 1);
    T2 u[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) u[n1] = line[n1];
    reg_fft<T, T2, N1>(u, a.dir);
#pragma unroll
    for (int i = 0; i < N1; ++i) {
      const int k = k2 + N2 * bit_reverse<N1>(i);   // output position
      int e = k + a.out_off;                          // stored entry
      if (e >= N) e -= N;
      if (e < a.out_cnt && !beyond_out(a, ia, b0 + j, e))
        outb[(int64_t)(b0 + j) * a.out_sb + (int64_t)e * a.out_se] = u[i];
    }
  }
}

// The forward x pass fused with combine_kernel's work: a workgroup transforms
// a run of lines of one grid in both interlaced copies and writes
// (D1 + e^{i pi (nx+ny+nz)/N} D2)/2 / W(n), minus the box-mode mean term, with
// the DC mode of dn_0^0 zeroed in box mode, straight into the spectra (the
// arithmetic of combine_kernel on the same FP32 transform outputs), so the
// copies' x-pass output never reaches HBM. The copies go through the same LDS
// one after the other; each thread keeps its first-copy outputs in registers
// (one step-C task per thread: lpw N2 <= the workgroup size). Lines: (grid,
// n_y, n_z) with n_z consecutive in a workgroup; stored entry e of an axis
// holds frequency e - R.
template <typename T, int N1, int N2>
__global__ void __launch_bounds__(kBlock) fft4_combine_kernel(PassArgs<T> a) {
  typedef typename cplx<T>::type T2;
  constexpr int N = N1 * N2;
  constexpr int LS = N2 * (N1 + 1) + 1;
  extern __shared__ char smem[];
  const int R = a.out_off, P = a.out_cnt;
  double* tab = (double*)smem;            // [3][P]: 1/W, cos and sin of pi n/N per axis entry
  T2* lds = (T2*)(smem + ((size_t)3 * P * sizeof(double) + 15) / 16 * 16);   // [line][LS]
  const int nbb = (a.dB + a.lpw - 1) / a.lpw;
  const int64_t blk = blockIdx.x;
  const int bb = (int)(blk % nbb);
  const int64_t rest = blk / nbb;
  const int ia = (int)(rest % a.dA);
  const int g = (int)(rest / a.dA);
  int b0 = bb * a.lpw;
  int nl = min(a.lpw, a.dB - b0);
  if (a.so_on) {   // lines beyond the band limit are never read: skip them (uniform)
    const int64_t rem = a.so_r2 - (int64_t)(ia - a.so_a) * (ia - a.so_a);
    if (rem < 0) return;
    int h = (int)sqrt((double)rem);
    while ((int64_t)h * h > rem) --h;
    while ((int64_t)(h + 1) * (h + 1) <= rem) ++h;
    const int lo = max(b0, a.so_b - h), hi = min(b0 + nl, a.so_b + h + 1);
    if (lo >= hi) return;
    b0 = lo;
    nl = hi - lo;
  }
  const int nc = a.cb_copies;
  const int tid = threadIdx.x;
  for (int i = tid; i < 3 * P; i += kBlock) tab[i] = a.cb_tab[i];   // read after the barriers below
  const bool has_task = tid < nl * N2;
  const int k2 = tid / nl, j = tid - (tid / nl) * nl;   // this thread's step-C task
  T2 u[N1], u2[N1];
  // step-A task of this thread (lpw N1 <= lpw N2 <= kBlock: at most one). For
  // lines of up to 256 points the inputs of both copies are loaded at once, so
  // the second copy's loads are in flight while the first copy is transformed
  // (longer lines would hold too many registers).
  constexpr bool kBoth = N2 <= 16;
  const bool has_a = tid < nl * N1;
  const int n1a = tid / nl, jja = tid - (tid / nl) * nl;
  auto load_a = [&](int c, T2 (&v)[N2]) {
    const T2* src = a.in + (int64_t)g * a.in_bs + (int64_t)c * a.cb_copy_bs + (int64_t)ia * a.in_sa +
                    (int64_t)(b0 + jja) * a.in_sb;
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) v[n2] = src[(int64_t)(n1a + N1 * n2) * a.in_se];
  };
  T2 va[kBoth ? 2 : 1][N2];
  if (kBoth && has_a) {
    load_a(0, va[0]);
    if (nc == 2) load_a(1, va[kBoth ? 1 : 0]);
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    if (c >= nc) break;
    if (c) __syncthreads();   // the first copy's step C has read the LDS
    // ---- step A: N2-point transforms of the copy's lines ---------------------
    if (has_a) {
      T2 (&v)[N2] = va[kBoth ? c : 0];
      if (!kBoth) load_a(c, v);
      reg_fft<T, T2, N2>(v, a.dir);
      T2* line = lds + jja * LS;
#pragma unroll
      for (int i = 0; i < N2; ++i) {
        const int kk = bit_reverse<N2>(i);
        T2 w = a.tw[(n1a * kk) % N];
        if (a.dir > 0) w.y = -w.y;
        T2 o;
        o.x = v[i].x * w.x - v[i].y * w.y;
        o.y = v[i].x * w.y + v[i].y * w.x;
        line[kk * (N1 + 1) + n1a] = o;
      }
    }
    __syncthreads();
    // ---- step C: N1-point transforms across n1 -----------------------------------
    if (has_task) {
      const T2* line = lds + j * LS + k2 * (N1 + 1);
      if (c == 0) {
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) u[n1] = line[n1];
        reg_fft<T, T2, N1>(u, a.dir);
      } else {
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) u2[n1] = line[n1];
        reg_fft<T, T2, N1>(u2, a.dir);
      }
    }
  }
  if (!has_task) return;
  // ---- the combination ----------------------------------------------------------
  const double* iw = tab;
  const double* pc = tab + P;
  const double* ps = tab + 2 * P;
  const double mean = a.cb_yspec ? a.cb_scal->mean_cell : 0.0;
  const int iy = ia, iz = b0 + j;
  const double czz = pc[iz], szz = ps[iz], wz = iw[iz];
  const double cy = pc[iy], sy = ps[iy], wy = iw[iy];
#pragma unroll
  for (int i = 0; i < N1; ++i) {
    const int k = k2 + N2 * bit_reverse<N1>(i);
    int ix = k + R;
    if (ix >= N) ix -= N;
    if (ix >= P || beyond_out(a, ia, iz, ix)) continue;
    const int64_t o_at = (int64_t)ix * a.out_se + (int64_t)iy * a.out_sa + (int64_t)iz * a.out_sb;
    double re = u[i].x, im = u[i].y;
    if (nc == 2) {
      const double cxy = pc[ix] * cy - ps[ix] * sy, sxy = pc[ix] * sy + ps[ix] * cy;
      const double cc = cxy * czz - sxy * szz, sn = cxy * szz + sxy * czz;
      re = 0.5 * (re + cc * (double)u2[i].x - sn * (double)u2[i].y);
      im = 0.5 * (im + cc * (double)u2[i].y + sn * (double)u2[i].x);
    }
    const double inv_w = iw[ix] * wy * wz;
    re *= inv_w;
    im *= inv_w;
    if (a.cb_yspec) {
      const T2 y = a.cb_yspec[(int64_t)g * a.out_bs + o_at];
      re -= mean * (double)y.x;
      im -= mean * (double)y.y;
    }
    if (a.cb_box && g == 0 && ix == R && iy == R && iz == R) re = 0.0;
    T2 o;
    o.x = (T)re;
    o.y = (T)im;
    a.out[(int64_t)g * a.out_bs + o_at] = o;
  }
}

template <typename T, int N1, int N2>
int launch_fft4_combine(PassArgs<T>& a, hipStream_t s, int lpw_req) {
  typedef typename cplx<T>::type T2;
  constexpr int LS = N2 * (N1 + 1) + 1;
  // lines per workgroup: one step-C task per thread (lpw N2 <= kBlock), at most
  // 40 KiB of LDS by default, a tuned value within 64 KiB
  const int64_t per_line = LS * (int64_t)sizeof(T2);
  const int64_t tab_bytes = ((int64_t)3 * a.out_cnt * 8 + 15) / 16 * 16;
  int lpw = kBlock / N2;
  while (lpw > 1 && lpw * per_line > 40 * 1024) lpw /= 2;
  if (lpw_req > 0) {
    lpw = std::min(lpw_req, kBlock / N2);
    while (lpw > 1 && lpw * per_line > 64 * 1024) lpw /= 2;
  }
  a.lpw = lpw;
  const int64_t nbb = (a.dB + a.lpw - 1) / a.lpw;
  const int64_t blocks = (int64_t)a.nbatch * a.dA * nbb;
  if (blocks > 2147483647LL) return fail(TSB_E_UNSUPPORTED, "FFT pass too large");
  hipLaunchKernelGGL((fft4_combine_kernel<T, N1, N2>), dim3((unsigned)blocks), dim3(kBlock),
                     (size_t)(tab_bytes + lpw * per_line), s, a);
  return TSB_OK;
}

template <typename T>
int launch_combine_pass(Plan& P, int stage, PassArgs<T>& a, hipStream_t s) {
  if (a.nbatch <= 0 || a.dA <= 0 || a.dB <= 0) return TSB_OK;
  prof_begin(P, stage, s);
  int rc = TSB_OK;
  const int req = P.lpw_tune[stage];
  switch (a.N) {
    case 16: rc = launch_fft4_combine<T, 4, 4>(a, s, req); break;
    case 32: rc = launch_fft4_combine<T, 4, 8>(a, s, req); break;
    case 64: rc = launch_fft4_combine<T, 8, 8>(a, s, req); break;
    case 128: rc = launch_fft4_combine<T, 8, 16>(a, s, req); break;
    case 256: rc = launch_fft4_combine<T, 16, 16>(a, s, req); break;
    case 512: rc = launch_fft4_combine<T, 16, 32>(a, s, req); break;
    default: rc = launch_fft4_combine<T, 32, 32>(a, s, req); break;
  }
  prof_end(P, stage, s);
  if (rc) return rc;
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

int pick_lpw(int N, int esz) {
  // two LDS line buffers of (N+1) complex each, at most 64 KiB
  int lpw = 16;
  while (lpw > 1 && (int64_t)2 * lpw * (N + 1) * 2 * esz > 65536) lpw /= 2;
  return lpw;
}

template <typename T, int N1, int N2>
int launch_fft4(PassArgs<T>& a, hipStream_t s, int lpw_req) {
  typedef typename cplx<T>::type T2;
  constexpr int LS = N2 * (N1 + 1) + 1;
  // lines per workgroup: the largest power of two up to 64 whose LDS stays
  // within 40 KiB, or a tuned value (at most 64 KiB of LDS)
  int lpw = 64;
  while (lpw > 1 && (int64_t)lpw * LS * (int64_t)sizeof(T2) > 40 * 1024) lpw /= 2;
  if (lpw_req > 0) {
    lpw = lpw_req;
    while (lpw > 1 && (int64_t)lpw * LS * (int64_t)sizeof(T2) > 64 * 1024) lpw /= 2;
  }
  a.lpw = lpw;
  const int64_t nbb = (a.dB + a.lpw - 1) / a.lpw;
  const int64_t blocks = (int64_t)a.nbatch * a.dA * nbb;
  if (blocks > 2147483647LL) return fail(TSB_E_UNSUPPORTED, "FFT pass too large");
  const size_t lds = (size_t)lpw * LS * sizeof(T2);
  hipLaunchKernelGGL((fft4_kernel<T, N1, N2>), dim3((unsigned)blocks), dim3(kBlock), lds, s, a);
  return TSB_OK;
}

template <typename T>
int launch_pass(Plan& P, int stage, PassArgs<T>& a, hipStream_t s) {
  typedef typename cplx<T>::type T2;
  if (a.nbatch <= 0 || a.dA <= 0 || a.dB <= 0) return TSB_OK;
  prof_begin(P, stage, s);
  int rc = TSB_OK;
  const int req = P.lpw_tune[stage];
  switch (a.N) {
    case 16: rc = launch_fft4<T, 4, 4>(a, s, req); break;
    case 32: rc = launch_fft4<T, 4, 8>(a, s, req); break;
    case 64: rc = launch_fft4<T, 8, 8>(a, s, req); break;
    case 128: rc = launch_fft4<T, 8, 16>(a, s, req); break;
    case 256: rc = launch_fft4<T, 16, 16>(a, s, req); break;
    case 512: rc = launch_fft4<T, 16, 32>(a, s, req); break;
    case 1024: rc = launch_fft4<T, 32, 32>(a, s, req); break;
    default: {
      // lengths with a factor 3: LDS Stockham radix 4/2/3
      a.lpw = pick_lpw(a.N, sizeof(T));
      const int64_t nbb = (a.dB + a.lpw - 1) / a.lpw;
      const int64_t blocks = (int64_t)a.nbatch * a.dA * nbb;
      if (blocks > 2147483647LL) return fail(TSB_E_UNSUPPORTED, "FFT pass too large");
      const size_t lds = (size_t)2 * a.lpw * (a.N + 1) * sizeof(T2);
      hipLaunchKernelGGL(fft_pass_kernel<T>, dim3((unsigned)blocks), dim3(kBlock), lds, s, a);
    }
  }
  prof_end(P, stage, s);
  if (rc) return rc;
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

int grid_blocks(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  return (int)(b < 1 ? 1 : b);
}

template <typename T>
int forward_impl(Plan& P, hipStream_t s) {
  typedef typename cplx<T>::type T2;
  const int N = P.N, PG = P.PG, RG = P.RG;
  const int64_t PGs = pad_line(PG);   // stored innermost extent of the pass buffers
  const int nbc = P.copies * (int)P.grids.size();
  const int64_t N2 = (int64_t)N * N, N3 = N2 * N;
  int rc;
  // Band limit of the spectra: with the reduced-grid rule nothing beyond
  // |n|^2 = n2maxG is read (the G chain masks it, the F cube and the shells
  // lie inside), so the y pass does not write the (n_y, n_z) entries beyond it
  // and the fused x pass neither transforms those lines nor writes beyond it.
  auto band = [&](PassArgs<T>& a, int oa, int ob, int oe) {
    if (P.n2maxG < 0) return;
    a.so_on = 1;
    a.so_r2 = P.n2maxG;
    a.so_a = oa;
    a.so_b = ob;
    a.so_e = oe;
  };
  // z (contiguous): [nbc][N][N][N] -> [nbc][N][N][PG], unless the column
  // assignment has just written its output
  const bool zdone = P.zcol_pass != 0;
  P.zcol_pass = 0;
  if (!zdone) {
    PassArgs<T> a{};
    a.in = (const T2*)P.d_grid;
    a.out = (T2*)P.d_t1;
    a.tw = (const T2*)P.d_tw_n;
    a.nbatch = nbc; a.dA = N; a.dB = N;
    a.in_bs = N3; a.in_sa = N2; a.in_sb = N; a.in_se = 1;
    a.out_bs = N2 * PGs; a.out_sa = (int64_t)N * PGs; a.out_sb = PGs; a.out_se = 1;
    a.in_cnt = N; a.in_off = 0; a.out_cnt = PG; a.out_off = RG;
    a.N = N; a.dir = -1; a.contiguous = 1;
    if ((rc = launch_pass<T>(P, kStFwdZ, a, s))) return rc;
  }
  // y (strided): [nbc][N][N][PG] -> [nbc][N][PG][PG]
  {
    PassArgs<T> a{};
    a.in = (const T2*)P.d_t1;
    a.out = (T2*)P.d_t2;
    a.tw = (const T2*)P.d_tw_n;
    a.nbatch = nbc; a.dA = N; a.dB = PG;
    a.in_bs = N2 * PGs; a.in_sa = (int64_t)N * PGs; a.in_sb = 1; a.in_se = PGs;
    a.out_bs = (int64_t)N * PG * PGs; a.out_sa = (int64_t)PG * PGs; a.out_sb = 1; a.out_se = PGs;
    a.in_cnt = N; a.in_off = 0; a.out_cnt = PG; a.out_off = RG;
    a.N = N; a.dir = -1; a.contiguous = 0;
    if (combine_fusable(N)) band(a, -1, RG, RG);   // (n_y, n_z) beyond the band: the fused x pass skips the line
    if ((rc = launch_pass<T>(P, kStFwdY, a, s))) return rc;
  }
  // x (strided): [nbc][N][PG][PG] -> [nbc][PG][PG][PG], or for the
  // register-FFT lengths the x pass and the combination in one kernel:
  // [copies][ngrid][N][PG][PG] -> spectra [ngrid][PG][PG][PG]
  const bool fused_x = combine_fusable(N);
  {
    PassArgs<T> a{};
    a.in = (const T2*)P.d_t2;
    a.out = (T2*)P.d_t3;
    a.tw = (const T2*)P.d_tw_n;
    a.nbatch = nbc; a.dA = PG; a.dB = PG;
    a.in_bs = (int64_t)N * PG * PGs; a.in_sa = PGs; a.in_sb = 1; a.in_se = (int64_t)PG * PGs;
    a.out_bs = (int64_t)PG * PG * PG; a.out_sa = PG; a.out_sb = 1; a.out_se = (int64_t)PG * PG;
    a.in_cnt = N; a.in_off = 0; a.out_cnt = PG; a.out_off = RG;
    a.N = N; a.dir = -1; a.contiguous = 0;
    if (fused_x) {
      band(a, RG, RG, RG);
      a.nbatch = (int)P.grids.size();
      a.out = (T2*)(P.wpass ? P.d_nspec : P.d_spec);
      a.cb_copies = P.copies;
      a.cb_copy_bs = (int64_t)P.grids.size() * a.in_bs;
      a.cb_tab = (const double*)P.d_axis_tab;
      a.cb_yspec = (!P.wpass && P.yspec_ready) ? (const T2*)P.d_yspec : nullptr;
      a.cb_scal = P.wpass ? (const DevScalars*)P.d_scal_n : (const DevScalars*)P.d_scal;
      a.cb_box = P.wpass ? 0 : P.box_mode;
      if ((rc = launch_combine_pass<T>(P, kStFwdX, a, s))) return rc;
    } else if ((rc = launch_pass<T>(P, kStFwdX, a, s))) {
      return rc;
    }
  }
  prof_begin(P, kStCombine, s);
  const int64_t row_pairs = ((int64_t)P.grids.size() * PG * PG + 1) / 2;   // two rows per workgroup
  if (P.wpass) {
    // the w^2-weighted N fields of the shot noise: a pure particle sum (no mean
    // term, DC kept), into their own spectra
    if (!fused_x) {
      hipLaunchKernelGGL(combine_kernel<T>, dim3((int)std::min<int64_t>(row_pairs, 8192)), dim3(kBlock), 0, s,
                         (const T2*)P.d_t3, (T2*)P.d_nspec, (int)P.grids.size(), P.copies, RG, 0,
                         (const double*)P.d_axis_tab, (const T2*)nullptr, (const DevScalars*)P.d_scal_n);
    }
    prof_end(P, kStCombine, s);
    TSB_HIP(hipGetLastError());
    return TSB_OK;
  }
  if (!fused_x) {
    hipLaunchKernelGGL(combine_kernel<T>, dim3((int)std::min<int64_t>(row_pairs, 8192)), dim3(kBlock), 0, s,
                       (const T2*)P.d_t3, (T2*)P.d_spec, (int)P.grids.size(), P.copies, RG, P.box_mode,
                       (const double*)P.d_axis_tab, P.yspec_ready ? (const T2*)P.d_yspec : (const T2*)nullptr,
                       (const DevScalars*)P.d_scal);
  }
  const int64_t pf3 = (int64_t)P.PF * P.PF * P.PF;
  hipLaunchKernelGGL(dcube_kernel<T>, dim3(grid_blocks(pf3)), dim3(kBlock), 0, s, (const T2*)P.d_spec,
                     (T2*)P.d_dcube, RG, P.RF);
  prof_end(P, kStCombine, s);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

// One inverse 3D transform chain on the M grid, from a cube of half-width R
// (stored entries 2R+1 per axis, [qx][qy][qz]) to full complex fields
// [nbatch][M^3]. Order x, y, z: the last and largest pass runs along the
// contiguous axis.
template <typename T>
int inverse_chain(Plan& P, int stage0, const typename cplx<T>::type* cube, int64_t cube_bs, int nbatch,
                  int R, PassArgs<T> pre, typename cplx<T>::type* fields, bool last_pass, hipStream_t s) {
  typedef typename cplx<T>::type T2;
  const int M = P.M, PR = 2 * R + 1;
  const int64_t M2 = (int64_t)M * M, PR2 = (int64_t)PR * PR, PRs = pad_line(PR);
  int rc;
  // Sparsity: shell-filtered slots vanish outside the largest |n|^2 of their
  // bin, band-limited grids outside n2max; lines beyond them are skipped.
  PassArgs<T> sp{};
  if (pre.pre == 2 || pre.pre == 4) {
    sp.sp = 1;
    sp.sp_r2 = P.d_bin_r2;
    sp.sp_div = pre.nkinds;
  } else if (pre.pre == 1) {
    sp.sp = 1;
    sp.sp_c = pre.n2max;
    sp.sp_div = 1;
  }
  auto sparse = [&](PassArgs<T>& a, int oa, int ob, int oe) {
    a.sp = sp.sp;
    a.sp_r2 = sp.sp_r2;
    a.sp_div = sp.sp_div;
    a.sp_c = sp.sp_c;
    a.sp_a = oa;
    a.sp_b = ob;
    a.sp_e = oe;
  };
  // x with the pre-operation: [b][qx][qy][qz] -> [b][x][qy][qz]
  {
    PassArgs<T> a = pre;
    sparse(a, R, R, R);
    a.in = cube;
    a.out = (T2*)P.d_u1;
    a.tw = (const T2*)P.d_tw_m;
    a.nbatch = nbatch; a.dA = PR; a.dB = PR;
    a.in_bs = cube_bs; a.in_sa = PR; a.in_sb = 1; a.in_se = PR2;
    a.out_bs = (int64_t)M * PR * PRs; a.out_sa = PRs; a.out_sb = 1; a.out_se = PR * PRs;
    a.in_cnt = PR; a.in_off = R; a.out_cnt = M; a.out_off = 0;
    a.offA = R; a.offB = R; a.offE = R;
    a.axA = 1; a.axB = 2; a.axE = 0;
    a.N = M; a.dir = 1; a.contiguous = 0;
    if ((rc = launch_pass<T>(P, stage0, a, s))) return rc;
  }
  // y: [b][x][qy][qz] -> [b][x][y][qz]
  {
    PassArgs<T> a{};
    a.in = (const T2*)P.d_u1;
    a.out = (T2*)P.d_u2;
    a.tw = (const T2*)P.d_tw_m;
    a.nbatch = nbatch; a.dA = M; a.dB = PR;
    a.in_bs = (int64_t)M * PR * PRs; a.in_sa = PR * PRs; a.in_sb = 1; a.in_se = PRs;
    a.out_bs = M2 * PRs; a.out_sa = (int64_t)M * PRs; a.out_sb = 1; a.out_se = PRs;
    a.in_cnt = PR; a.in_off = R; a.out_cnt = M; a.out_off = 0;
    a.N = M; a.dir = 1; a.contiguous = 0;
    sparse(a, -1, R, R);
    if ((rc = launch_pass<T>(P, stage0 + 1, a, s))) return rc;
  }
  // z (contiguous): [b][x][y][qz] -> [b][x][y][z]
  if (last_pass) {
    PassArgs<T> a{};
    a.in = (const T2*)P.d_u2;
    a.out = fields;
    a.tw = (const T2*)P.d_tw_m;
    a.nbatch = nbatch; a.dA = M; a.dB = M;
    a.in_bs = M2 * PRs; a.in_sa = (int64_t)M * PRs; a.in_sb = PRs; a.in_se = 1;
    a.out_bs = M2 * M; a.out_sa = M2; a.out_sb = M; a.out_se = 1;
    a.in_cnt = PR; a.in_off = R; a.out_cnt = M; a.out_off = 0;
    a.N = M; a.dir = 1; a.contiguous = 1;
    sparse(a, -1, -1, R);
    if ((rc = launch_pass<T>(P, stage0 + 2, a, s))) return rc;
  }
  return TSB_OK;
}

template <typename T>
int inverse_impl(Plan& P, hipStream_t s) {
  typedef typename cplx<T>::type T2;
  const int64_t M3 = (int64_t)P.M * P.M * P.M;
  const int nf = P.nb * (int)P.fkinds.size();
  T2* fields = (T2*)P.d_fields;
  int rc;
  // G grids first: band-limited spectra (eq. 42). The F chain runs last so that,
  // with the fused reduction, its y-pass output is still in d_u2 afterwards.
  // (The LOS at the first or second vertex needs G_0^0 only: grid 0.)
  {
    PassArgs<T> pre{};
    pre.pre = P.n2maxG >= 0 ? 1 : 0;
    pre.n2max = P.n2maxG;
    const int64_t pg3 = (int64_t)P.PG * P.PG * P.PG;
    // the shot noise's i = j != k term takes the H spectra in place of dn_L^M
    const void* gsrc = P.spass ? P.d_hspec : P.d_spec;
    const int ngi = P.g00_only ? 1 : (int)P.grids.size();
    if ((rc = inverse_chain<T>(P, kStInvGX, (const T2*)gsrc, pg3, ngi, P.RG, pre, fields + P.g_offset, true, s)))
      return rc;
  }
  if (P.spass && P.d_kslot) return TSB_OK;   // the 3PCF's shot-noise term needs the H fields only
  // F slots: shell filter of dn_0^0 times y_l^m*(k^) (eq. 42), or for the 3PCF
  // dn_0^0 times the slot's separation kernel (eq. 48)
  {
    PassArgs<T> pre{};
    pre.pre = P.d_kslot ? 3 : (P.fsources ? 4 : 2);
    pre.kslot = P.d_kslot;
    pre.kslot_bs = (int64_t)P.PF * P.PF * P.PF;
    pre.spec = P.d_spec;
    pre.RG = P.RG;
    pre.bin_lut = P.d_bin_lut;
    pre.lut_max = (int64_t)P.bin_lut.size() - 1;
    pre.kinds = P.d_fkinds;
    pre.nkinds = (int)P.fkinds.size();
    ylm_norm_table(pre.ynorm);
    // with the fused reduction the z pass of F happens inside the reduction
    // (the shot noise's unit shell fields f_l^m filter a cube of ones)
    const void* fsrc = P.spass ? P.d_ucube : P.d_dcube;
    if ((rc = inverse_chain<T>(P, kStInvFX, (const T2*)fsrc, 0, nf, P.RF, pre, fields, !P.fused, s)))
      return rc;
  }
  return TSB_OK;
}

// Separation kernels of the 3PCF (Sec. 4.3): for F slot (bin b, kind k) with
// parts (l_p, m_p, c_p),
//   Kslot(k) = sum_p c_p i^-l_p sum_{n in b} y_lp^mp*(n^) e^{2 pi i k.n / N},
// i.e. N_r(b) i^-l K_l^m(k; b) of eq. 49 on the grid. The sum over separation
// vectors is the inverse transform of the shell-filtered cube of ones with n in
// the role of the mode (the r-bin table maps n^2 to bins); the zero
// separation, which the shell filter skips, adds c_p for l_p = 0 to every mode
// when a bin holds r = 0.
template <typename T>
__global__ void __launch_bounds__(kBlock) kslot_gather_kernel(const typename cplx<T>::type* fields,
                                                             typename cplx<T>::type* kslot, int nbatch, int nkinds,
                                                             int N, int R, int zero_bin, const FKind* kinds) {
  typedef typename cplx<T>::type T2;
  const int PR = 2 * R + 1;
  const int64_t pr3 = (int64_t)PR * PR * PR, total = (int64_t)nbatch * pr3, N3 = (int64_t)N * N * N;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
    const int batch = (int)(i / pr3);
    const int64_t q = i - (int64_t)batch * pr3;
    const int qx = (int)(q / ((int64_t)PR * PR)), qy = (int)((q / PR) % PR), qz = (int)(q % PR);
    int x = qx - R, y = qy - R, z = qz - R;
    x += x < 0 ? N : 0;
    y += y < 0 ? N : 0;
    z += z < 0 ? N : 0;
    T2 v = fields[(int64_t)batch * N3 + ((int64_t)x * N + y) * N + z];
    if (batch / nkinds == zero_bin) {
      const FKind& k = kinds[batch % nkinds];
      for (int p = 0; p < k.nparts; ++p)
        if (k.part[p].l == 0) {
          v.x += (T)k.part[p].fr;
          v.y += (T)k.part[p].fi;
        }
    }
    kslot[i] = v;
  }
}

template <typename T>
int separation_impl(Plan& P, hipStream_t s) {
  typedef typename cplx<T>::type T2;
  if (P.M != P.N) return fail(TSB_E_UNSUPPORTED, "separation kernels need the reduction grid M = N");
  const int nk = (int)P.fkinds.size(), nf = P.nb * nk, PF = P.PF;
  const int64_t pf3 = (int64_t)PF * PF * PF, N3 = (int64_t)P.N * P.N * P.N;
  // slot kinds with the factors i^-l_p
  std::vector<FKind> kinds = P.fkinds;
  for (auto& k : kinds)
    for (int p = 0; p < k.nparts; ++p) {
      static const double ire[4] = {1, 0, -1, 0}, iim[4] = {0, -1, 0, 1};   // i^-l
      const int l4 = k.part[p].l % 4;
      const double fr = k.part[p].fr, fi = k.part[p].fi;
      k.part[p].fr = fr * ire[l4] - fi * iim[l4];
      k.part[p].fi = fr * iim[l4] + fi * ire[l4];
    }
  std::vector<T> ones(2 * pf3, (T)0);
  for (int64_t i = 0; i < pf3; ++i) ones[2 * i] = (T)1;
  void *d_kinds = nullptr, *d_ones = nullptr, *d_fields = nullptr;
  auto release = [&]() {
    if (d_kinds) (void)hipFree(d_kinds);
    if (d_ones) (void)hipFree(d_ones);
    if (d_fields) (void)hipFree(d_fields);
  };
  int rc = TSB_OK;
  if (hipMalloc(&d_kinds, kinds.size() * sizeof(FKind)) != hipSuccess ||
      hipMalloc(&d_ones, ones.size() * sizeof(T)) != hipSuccess ||
      hipMalloc(&d_fields, (size_t)nf * N3 * sizeof(T2)) != hipSuccess) {
    (void)hipGetLastError();
    release();
    return fail(TSB_E_NOMEM, "device allocation for the separation kernels failed");
  }
  if (hipMemcpy(d_kinds, kinds.data(), kinds.size() * sizeof(FKind), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d_ones, ones.data(), ones.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    release();
    return fail(TSB_E_DEVICE, "upload of the separation-kernel tables failed");
  }
  PassArgs<T> pre{};
  pre.pre = 2;
  pre.bin_lut = P.d_bin_lut;
  pre.lut_max = (int64_t)P.bin_lut.size() - 1;
  pre.kinds = (const FKind*)d_kinds;
  pre.nkinds = nk;
  ylm_norm_table(pre.ynorm);
  const unsigned saved = P.prof;
  P.prof = 0;
  rc = inverse_chain<T>(P, kStInvFX, (const T2*)d_ones, 0, nf, P.RF, pre, (T2*)d_fields, true, s);
  P.prof = saved;
  if (!rc) {
    hipLaunchKernelGGL(kslot_gather_kernel<T>, dim3(grid_blocks((int64_t)nf * pf3)), dim3(kBlock), 0, s,
                       (const T2*)d_fields, (T2*)P.d_kslot, nf, nk, P.N, P.RF, P.bin_lut[0], (const FKind*)d_kinds);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      rc = fail(TSB_E_DEVICE, "separation-kernel construction failed");
  }
  release();
  return rc;
}

}  // namespace

int run_inverse_cube(Plan& P, const void* cube, int nbatch, void* out, hipStream_t s) {
  const int64_t pg3 = (int64_t)P.PG * P.PG * P.PG;
  if (P.precision == TSB_FP64) {
    PassArgs<double> pre{};
    return inverse_chain<double>(P, kStInvGX, (const double2*)cube, pg3, nbatch, P.RG, pre, (double2*)out, true, s);
  }
  PassArgs<float> pre{};
  return inverse_chain<float>(P, kStInvGX, (const float2*)cube, pg3, nbatch, P.RG, pre, (float2*)out, true, s);
}

bool combine_fusable(int N) {
  return N == 16 || N == 32 || N == 64 || N == 128 || N == 256 || N == 512 || N == 1024;
}

int run_separation_kernels(Plan& P, hipStream_t s) {
  if (!P.d_kslot) return TSB_OK;
  return P.precision == TSB_FP64 ? separation_impl<double>(P, s) : separation_impl<float>(P, s);
}

int run_forward(Plan& P, hipStream_t s) {
  return P.precision == TSB_FP64 ? forward_impl<double>(P, s) : forward_impl<float>(P, s);
}

int run_inverse(Plan& P, hipStream_t s) {
  return P.precision == TSB_FP64 ? inverse_impl<double>(P, s) : inverse_impl<float>(P, s);
}

}  // namespace tsb
