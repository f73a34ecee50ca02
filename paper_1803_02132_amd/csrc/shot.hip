// Shot noise of the bispectrum multipoles (Sec. 4.2, eqs. 43-46).
//
// In the particle description (eq. 43) the estimator is a triple sum over
// particles i, j, k; the shot noise is its part with coincident indices
// (eq. 44), whose four terms (eq. 45) are built from the scalars
// Sbar_L^M = (sum_gal - alpha^3 sum_ran) w^3 y_L^M*(x^) and the w^2-weighted
// fields N_L^M(k) = (sum_gal + alpha^2 sum_ran) w^2 y_L^M(x^) e^{-ik.x} (eq. 46).
// With every shell average the discrete mode sum of eq. 38:
//   i = j = k:    (N H / I) sum_m 3j ybar_l1^m1*(b1) ybar_l2^m2*(b2) Sbar_L^M
//   j = k != i:   (N H / I) sum_m 3j A_{l1 m1}^{L M}(b1) ybar_l2^m2*(b2)
//   i = k != j:   (N H / I) sum_m 3j ybar_l1^m1*(b1) A_{l2 m2}^{L M}(b2)
//   i = j != k:   eq. 41 with F replaced by the unit shell fields
//                 f_l^m(x;b) = shell average of y_l^m*(k^) e^{ik.x} and G by
//                 H_L^M(x) = int d3k e^{ik.x} [dn_L^M N_0^0* - Sbar_L^M C/W^2]
// where A_{l m}^{L M}(b) = shell average of y_l^m*(k^) [dn N_L^M* - Sbar_L^M C/W^2]
// and C is the alias sum of W_mass^2 (the self-pair term of dn N* that the
// subtraction removes; per axis, closed forms of sum_n sinc^{2p}(x + pi n) and of
// the alternating sum, combined over the parity of the aliases when the grids
// are interlaced).
//
// The N channels go through the assignment and forward transforms as a second
// pass with weights w^2 (plan field wpass); this file holds the k-space
// kernels (H spectra on the G cube, the shell sums on the F cube) and the host
// side: the tables made at plan creation and the final combination.
#include <algorithm>
#include <cmath>
#include <limits>
#include <map>
#include <tuple>

#include "tsb_internal.h"

namespace tsb {

namespace {

// N_L^M*(n) at stored cube index n (and -n) of the combined N spectra, for any
// M, from the complex grids: srcg = grid, kind 0 = the grid holds the complex
// channel (L, |M|) (M != 0), 1 = the real channel (L, 0) in the grid's real
// slot, 2 = in its imaginary slot. Writing Nt_L^M for the y*-weighted w^2 field
// (the same convention as dn_L^M): N_L^M*(k) = Nt_L^M(-k), and for M < 0,
// Nt_L^M(k) = (-1)^M conj(Nt_L^|M|(-k)).
struct LMSrc { int grid, kind, M; };

template <typename T2>
__device__ inline double2 ld(const T2* p, int64_t i) {
  const T2 v = p[i];
  return make_double2((double)v.x, (double)v.y);
}

template <typename T2>
__device__ inline double2 nt_at(const T2* spec, int64_t P3, const LMSrc& s, int64_t ip, int64_t im) {
  // Nt_L^|M| at +n (index ip); -n has index im
  const T2* g = spec + (int64_t)s.grid * P3;
  const double2 a = ld(g, ip);
  if (s.kind == 0) return a;
  const double2 b = ld(g, im);
  if (s.kind == 1) return make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));   // (Z(n) + conj Z(-n))/2
  return make_double2(0.5 * (a.y + b.y), -0.5 * (a.x - b.x));                     // (Z(n) - conj Z(-n))/(2i)
}

template <typename T2>
__device__ inline double2 nstar(const T2* spec, int64_t P3, const LMSrc& s, int64_t ip, int64_t im) {
  if (s.M >= 0) return nt_at(spec, P3, s, im, ip);   // Nt(-n)
  const double2 v = nt_at(spec, P3, s, ip, im);      // (-1)^|M| conj(Nt^|M|(n))
  const double sg = (s.M & 1) ? -1.0 : 1.0;
  return make_double2(sg * v.x, -sg * v.y);
}

// C(k)/W^2(k) at stored G-cube indices (ix, iy, iz): tab = [A_p | B_p] per axis
// entry, iw = 1/W per axis entry.
__device__ inline double cw2_at(const double* tab, const double* iw, int P, int ix, int iy, int iz, int interlace) {
  double c = tab[ix] * tab[iy] * tab[iz];
  if (interlace) c = 0.5 * (c + tab[P + ix] * tab[P + iy] * tab[P + iz]);
  const double w = iw[ix] * iw[iy] * iw[iz];
  return c * w * w;
}

struct HArgs {
  const void* spec;    // dn spectra [ngrid][PG^3]
  const void* nspec;   // N spectra [ngrid][PG^3]
  void* hspec;         // out [ngrid][PG^3]
  const double* sbar;  // per real channel
  const double* tab;   // A_p, B_p per G-cube axis entry
  const double* iw;    // 1/W per G-cube axis entry
  int RG, ngrid, interlace;
  int gre[32], gim[32];   // channels of each complex grid (-1: none)
  LMSrc n00;              // where Nt_0^0 sits
};

// H_L^M spectra per complex grid g (real channels re + i im): Z_g(n) N_0^0*(n)
// - (Sbar_re + i Sbar_im) C(n)/W^2(n); N_0^0 is a real field's transform, so the
// product keeps the two channels apart.
template <typename T>
__global__ void __launch_bounds__(kBlock) hspec_kernel(HArgs a) {
  typedef typename cplx<T>::type T2;
  const int P = 2 * a.RG + 1;
  const int64_t P3 = (int64_t)P * P * P;
  const T2* spec = (const T2*)a.spec;
  const T2* nspec = (const T2*)a.nspec;
  T2* out = (T2*)a.hspec;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (int64_t)a.ngrid * P3;
       i += (int64_t)gridDim.x * kBlock) {
    const int g = (int)(i / P3);
    const int64_t c = i - (int64_t)g * P3;
    const int ix = (int)(c / ((int64_t)P * P)), iy = (int)((c / P) % P), iz = (int)(c % P);
    const int64_t cm = ((int64_t)(P - 1 - ix) * P + (P - 1 - iy)) * P + (P - 1 - iz);   // -n
    const double2 z = ld(spec + (int64_t)g * P3, c);
    const double2 n = nstar(nspec, P3, a.n00, c, cm);
    const double cw = cw2_at(a.tab, a.iw, P, ix, iy, iz, a.interlace);
    const double sr = a.gre[g] >= 0 ? a.sbar[a.gre[g]] : 0.0, si = a.gim[g] >= 0 ? a.sbar[a.gim[g]] : 0.0;
    T2 o;
    o.x = (T)(z.x * n.x - z.y * n.y - sr * cw);
    o.y = (T)(z.x * n.y + z.y * n.x - si * cw);
    out[i] = o;
  }
}

struct SumArgs {
  const void* dcube;   // dn_0^0 on the F cube [PF^3]
  const void* nspec;   // N spectra on the G cube
  const double* sbar;
  const double* tab, *iw;
  const int* modes;    // F-cube linear indices, bin by bin
  const int* start;    // [nb + 1]
  const Plan::SnCombo* combos;
  int RF, RG, nb, interlace;
  double ynorm[45];
  LMSrc src[81];       // N source of (L, M), index L(L+1) + M (local) ; (0, 0) global
  int sre[81], sim[81];   // real channels of (L, |M|): Sbar_L^|M| = sbar[sre] + i sbar[sim]
  double* out;         // [combo][bin][2]
};

// One block per (combo, shell): sum over the shell's modes of
// y_l^m*(k^) [dn(k) N_L^M*(k) - Sbar_L^M C(k)/W^2(k)], a fixed-shape tree.
template <typename T>
__global__ void __launch_bounds__(kBlock) shell_sums_kernel(SumArgs a) {
  typedef typename cplx<T>::type T2;
  __shared__ double shr[kBlock], shi[kBlock];
  const int combo = blockIdx.x, b = blockIdx.y;
  const Plan::SnCombo cb = a.combos[combo];
  const int PF = 2 * a.RF + 1, PG = 2 * a.RG + 1;
  const int64_t PG3 = (int64_t)PG * PG * PG;
  const int li = cb.L * (cb.L + 1) + cb.M;
  const LMSrc src = a.src[li];
  const int aM = cb.M < 0 ? -cb.M : cb.M;
  const int lia = cb.L * (cb.L + 1) + aM;
  double sbr = a.sre[lia] >= 0 ? a.sbar[a.sre[lia]] : 0.0, sbi = a.sim[lia] >= 0 ? a.sbar[a.sim[lia]] : 0.0;
  if (cb.M < 0) {   // Sbar_L^M = (-1)^|M| conj(Sbar_L^|M|)
    const double sg = (aM & 1) ? -1.0 : 1.0;
    sbr *= sg;
    sbi *= -sg;
  }
  const T2* dc = (const T2*)a.dcube;
  const T2* ns = (const T2*)a.nspec;
  double accr = 0.0, acci = 0.0;
  for (int q = a.start[b] + threadIdx.x; q < a.start[b + 1]; q += kBlock) {
    const int i = a.modes[q];
    const int fx = i / (PF * PF) - a.RF, fy = (i / PF) % PF - a.RF, fz = i % PF - a.RF;
    const int ix = fx + a.RG, iy = fy + a.RG, iz = fz + a.RG;
    const int64_t cp = ((int64_t)ix * PG + iy) * PG + iz;
    const int64_t cm = ((int64_t)(PG - 1 - ix) * PG + (PG - 1 - iy)) * PG + (PG - 1 - iz);
    const double2 d = ld(dc, i);
    const double2 n = nstar(ns, PG3, src, cp, cm);
    const double cw = cw2_at(a.tab, a.iw, PG, ix, iy, iz, a.interlace);
    const double pr = d.x * n.x - d.y * n.y - sbr * cw, pi = d.x * n.y + d.y * n.x - sbi * cw;
    const double r = sqrt((double)fx * fx + (double)fy * fy + (double)fz * fz);
    double yr, yi;
    const int am = cb.m < 0 ? -cb.m : cb.m;
    ylm_pos_m(cb.l, am, fx / r, fy / r, fz / r, a.ynorm, &yr, &yi);
    // y_l^m* : (yr, -yi) for m >= 0; (-1)^|m| (yr, yi) for m < 0
    double ur = yr, ui = -yi;
    if (cb.m < 0) {
      const double sg = (am & 1) ? -1.0 : 1.0;
      ur = sg * yr;
      ui = sg * yi;
    }
    accr += ur * pr - ui * pi;
    acci += ur * pi + ui * pr;
  }
  shr[threadIdx.x] = accr;
  shi[threadIdx.x] = acci;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      shr[threadIdx.x] += shr[threadIdx.x + st];
      shi[threadIdx.x] += shi[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.out[((size_t)combo * a.nb + b) * 2] = shr[0];
    a.out[((size_t)combo * a.nb + b) * 2 + 1] = shi[0];
  }
}

struct SepArgs {
  const void* gfields;     // real-space fields of the H spectra [ngrid][N^3]
  const int* sep;          // F-cube indices of the separation vectors, bin by bin
  const int* start;        // [nb + 1]
  const OutEntry* outs;
  const QGroup* qg;
  const Term* terms;
  const Component* fcomp;
  const Component* gcomp;
  const FKind* kinds;
  const double* out_norm;
  const DevScalars* scal;
  double* B;
  int N, RF;
  double ynorm[45];
};

// Real or imaginary part of sum_p c_p i^-l_p y_lp^mp*(n^) for an F slot kind:
// the slot's separation kernel at the separation vector n, per unit weight
// (the zero separation has y_l^m = delta_l0).
__device__ inline double kind_at(const FKind& k, int part, bool zero, double ux, double uy, double uz,
                                 const double* ynorm) {
  double sr = 0.0, si = 0.0;
  for (int p = 0; p < k.nparts; ++p) {
    const FPart& fp = k.part[p];
    const int am = fp.m < 0 ? -fp.m : fp.m;
    double ur, ui;   // y_l^m*
    if (zero) {
      ur = fp.l == 0 ? 1.0 : 0.0;
      ui = 0.0;
    } else {
      double yr, yi;
      ylm_pos_m(fp.l, am, ux, uy, uz, ynorm, &yr, &yi);
      ur = yr;
      ui = -yi;
      if (fp.m < 0) {
        const double sg = (am & 1) ? -1.0 : 1.0;
        ur = sg * yr;
        ui = sg * yi;
      }
    }
    static constexpr double ire[4] = {1, 0, -1, 0}, iim[4] = {0, -1, 0, 1};   // i^-l
    const int l4 = fp.l & 3;
    const double cr = fp.fr * ire[l4] - fp.fi * iim[l4], ci = fp.fr * iim[l4] + fp.fi * ire[l4];
    sr += cr * ur - ci * ui;
    si += cr * ui + ci * ur;
  }
  return part ? si : sr;
}

// The 3PCF's i = j != k term (eq. 51). With the full separation kernels the
// kernel field of slot kind k in bin b is a comb of points: the inverse
// transform of sum_{n in b} Y_k(n) e^{2 pi i k.n / N} is N^3 Y_k(n) at node -n.
// The sum over cells of f f H then runs over the bin's separation vectors and
// vanishes unless b1 = b2. One block per output, a fixed-shape tree; the
// plan's terms, coefficients and output norms are those of the reduction.
template <typename T>
__global__ void __launch_bounds__(kBlock) separation_shot_kernel(SepArgs a) {
  typedef typename cplx<T>::type T2;
  __shared__ double sh[kBlock];
  const OutEntry e = a.outs[blockIdx.x];
  const int N = a.N, RF = a.RF, PF = 2 * RF + 1;
  const int64_t N3 = (int64_t)N * N * N;
  const T2* g = (const T2*)a.gfields;
  double acc = 0.0;
  if (e.b1 == e.b2 && e.q1 > e.q0) {
    const int t0 = a.qg[e.q0].t0, t1 = a.qg[e.q1 - 1].t1;
    for (int q = a.start[e.b1] + threadIdx.x; q < a.start[e.b1 + 1]; q += kBlock) {
      const int i = a.sep[q];
      const int nx = i / (PF * PF) - RF, ny = (i / PF) % PF - RF, nz = i % PF - RF;
      const bool zero = nx == 0 && ny == 0 && nz == 0;
      const double r = zero ? 1.0 : sqrt((double)nx * nx + (double)ny * ny + (double)nz * nz);
      const double ux = nx / r, uy = ny / r, uz = nz / r;
      const int jx = nx > 0 ? N - nx : -nx, jy = ny > 0 ? N - ny : -ny, jz = nz > 0 ? N - nz : -nz;
      const int64_t node = ((int64_t)jx * N + jy) * N + jz;
      for (int t = t0; t < t1; ++t) {
        const Term tm = a.terms[t];
        const Component c1 = a.fcomp[tm.f1], c2 = a.fcomp[tm.f2], cg = a.gcomp[tm.g];
        const double f1 = kind_at(a.kinds[c1.slot], c1.part, zero, ux, uy, uz, a.ynorm);
        const double f2 = kind_at(a.kinds[c2.slot], c2.part, zero, ux, uy, uz, a.ynorm);
        const T2 gv = g[(int64_t)cg.slot * N3 + node];
        acc += tm.coef * f1 * f2 * (double)(cg.part ? gv.y : gv.x);
      }
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double n3 = (double)N3;
    a.B[blockIdx.x] = sh[0] * n3 * n3 * a.out_norm[blockIdx.x] / a.scal->I;
  }
}

template <typename T>
int separation_shot_impl(Plan& P, hipStream_t s) {
  if (P.outs.empty()) return TSB_OK;
  SepArgs a{};
  a.gfields = (const typename cplx<T>::type*)P.d_fields + P.g_offset;
  a.sep = P.d_shell_modes;
  a.start = P.d_shell_start;
  a.outs = P.d_outs;
  a.qg = P.d_qgroups;
  a.terms = P.d_terms;
  a.fcomp = P.d_fcomp;
  a.gcomp = P.d_gcomp;
  a.kinds = P.d_fkinds;
  a.out_norm = P.d_out_norm;
  a.scal = P.d_scal;
  a.B = P.d_B;
  a.N = P.N;
  a.RF = P.RF;
  ylm_norm_table(a.ynorm);
  hipLaunchKernelGGL(separation_shot_kernel<T>, dim3((unsigned)P.outs.size()), dim3(kBlock), 0, s, a);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

// Two-point spectra of the 3PCF's j = k and i = k terms, for each (L, M) in
// the list: v(k) = dn(k) N_L^M*(k) - Sbar_L^M C(k)/W^2(k) on the F cube (which
// for the 3PCF is the whole grid without its Nyquist planes, where every field
// is zero).
constexpr int kMaxV = 81;
struct VArgs {
  const void* dcube;   // dn_0^0 on the F cube [PF^3]
  const void* nspec;   // N spectra on the G cube
  void* vspec;         // out [nv][PF^3]
  const double* sbar;
  const double* tab, *iw;
  int RF, RG, nv, interlace;
  LMSrc src[kMaxV];    // N source of each (L, M)
  short sre[kMaxV], sim[kMaxV], sgn[kMaxV];   // channels of Sbar_L^|M|; M < 0: (-1)^|M| conj
};

template <typename T>
__global__ void __launch_bounds__(kBlock) vspec_kernel(VArgs a) {
  typedef typename cplx<T>::type T2;
  const int PF = 2 * a.RF + 1, PG = 2 * a.RG + 1;
  const int64_t PF3 = (int64_t)PF * PF * PF, PG3 = (int64_t)PG * PG * PG;
  const T2* dc = (const T2*)a.dcube;
  const T2* ns = (const T2*)a.nspec;
  T2* out = (T2*)a.vspec;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (int64_t)a.nv * PF3;
       i += (int64_t)gridDim.x * kBlock) {
    const int v = (int)(i / PF3);
    const int64_t c = i - (int64_t)v * PF3;
    const int fx = (int)(c / ((int64_t)PF * PF)) - a.RF, fy = (int)((c / PF) % PF) - a.RF, fz = (int)(c % PF) - a.RF;
    const int ix = fx + a.RG, iy = fy + a.RG, iz = fz + a.RG;
    const int64_t cp = ((int64_t)ix * PG + iy) * PG + iz;
    const int64_t cm = ((int64_t)(PG - 1 - ix) * PG + (PG - 1 - iy)) * PG + (PG - 1 - iz);
    double sbr = a.sre[v] >= 0 ? a.sbar[a.sre[v]] : 0.0, sbi = a.sim[v] >= 0 ? a.sbar[a.sim[v]] : 0.0;
    if (a.sgn[v] != 0) {   // M < 0: Sbar_L^M = (-1)^|M| conj(Sbar_L^|M|)
      sbr *= a.sgn[v];
      sbi *= -a.sgn[v];
    }
    const double2 d = ld(dc, c);
    const double2 n = nstar(ns, PG3, a.src[v], cp, cm);
    const double cw = cw2_at(a.tab, a.iw, PG, ix, iy, iz, a.interlace);
    T2 o;
    o.x = (T)(d.x * n.x - d.y * n.y - sbr * cw);
    o.y = (T)(d.x * n.y + d.y * n.x - sbi * cw);
    out[i] = o;
  }
}

struct TwoArgs {
  const void* vfields;   // inverse transforms of the two-point spectra [nv][N^3]
  const int* sep;        // F-cube indices of the separation vectors, bin by bin
  const int* start;      // [nb + 1]
  const Plan::SnCombo* combos;
  int N, RF, nb;
  double ynorm[45];
  double* out;           // [combo][bin][2]
};

// Two-point sums of the 3PCF (the shell sums' counterpart): one block per
// (combo, bin), sum over the bin's separation vectors n of y_l^m*(n^) v(Hn)
// with v the inverse transform of the combo's two-point spectrum (node +n;
// the zero separation has y = delta_l0), a fixed-shape tree.
template <typename T>
__global__ void __launch_bounds__(kBlock) twopoint_sums_kernel(TwoArgs a, const int* combo_v) {
  typedef typename cplx<T>::type T2;
  __shared__ double shr[kBlock], shi[kBlock];
  const int combo = blockIdx.x, b = blockIdx.y;
  const Plan::SnCombo cb = a.combos[combo];
  const int N = a.N, RF = a.RF, PF = 2 * RF + 1;
  const int64_t N3 = (int64_t)N * N * N;
  const T2* vf = (const T2*)a.vfields + (int64_t)combo_v[combo] * N3;
  double accr = 0.0, acci = 0.0;
  for (int q = a.start[b] + threadIdx.x; q < a.start[b + 1]; q += kBlock) {
    const int i = a.sep[q];
    const int nx = i / (PF * PF) - RF, ny = (i / PF) % PF - RF, nz = i % PF - RF;
    double ur, ui;   // y_l^m*(n^)
    if (nx == 0 && ny == 0 && nz == 0) {
      ur = cb.l == 0 ? 1.0 : 0.0;
      ui = 0.0;
    } else {
      const double r = sqrt((double)nx * nx + (double)ny * ny + (double)nz * nz);
      const int am = cb.m < 0 ? -cb.m : cb.m;
      double yr, yi;
      ylm_pos_m(cb.l, am, nx / r, ny / r, nz / r, a.ynorm, &yr, &yi);
      ur = yr;
      ui = -yi;
      if (cb.m < 0) {
        const double sg = (am & 1) ? -1.0 : 1.0;
        ur = sg * yr;
        ui = sg * yi;
      }
    }
    const int jx = nx < 0 ? nx + N : nx, jy = ny < 0 ? ny + N : ny, jz = nz < 0 ? nz + N : nz;
    const T2 v = vf[((int64_t)jx * N + jy) * N + jz];
    accr += ur * (double)v.x - ui * (double)v.y;
    acci += ur * (double)v.y + ui * (double)v.x;
  }
  shr[threadIdx.x] = accr;
  shi[threadIdx.x] = acci;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      shr[threadIdx.x] += shr[threadIdx.x + st];
      shi[threadIdx.x] += shi[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.out[((size_t)combo * a.nb + b) * 2] = shr[0];
    a.out[((size_t)combo * a.nb + b) * 2 + 1] = shi[0];
  }
}

// Where Nt_L^|M| (and the channels of Sbar_L^|M|) sit in the plan's grids.
void lm_sources(const Plan& P, LMSrc* src, int* sre, int* sim) {
  for (int k = 0; k < 81; ++k) {
    src[k] = {0, 1, 0};
    sre[k] = sim[k] = -1;
  }
  for (int g = 0; g < (int)P.grids.size(); ++g) {
    for (int part = 0; part < 2; ++part) {
      const int c = part ? P.grids[g].im : P.grids[g].re;
      if (c < 0) continue;
      const RealChannel& ch = P.chans[c];
      const int li = ch.L * (ch.L + 1) + ch.M;
      if (ch.M == 0) {
        src[li] = {g, part ? 2 : 1, 0};
        sre[li] = c;
      } else {
        src[li] = {g, 0, ch.M};
        src[ch.L * (ch.L + 1) - ch.M] = {g, 0, -ch.M};
        (ch.part ? sim : sre)[li] = c;
      }
    }
  }
}

template <typename T>
int kspace_impl(Plan& P, hipStream_t s) {
  HArgs h{};
  h.spec = P.d_spec;
  h.nspec = P.d_nspec;
  h.hspec = P.d_hspec;
  h.sbar = P.d_sbar;
  h.tab = P.d_cw2_tab;
  h.iw = P.d_axis_tab;   // [0, PG): 1/W per axis entry
  h.RG = P.RG;
  h.ngrid = (int)P.grids.size();
  h.interlace = P.interlace;
  for (int g = 0; g < h.ngrid; ++g) {
    h.gre[g] = P.grids[g].re;
    h.gim[g] = P.grids[g].im;
  }
  SumArgs a{};
  lm_sources(P, a.src, a.sre, a.sim);
  h.n00 = a.src[0];
  const int64_t PG = P.PG;
  const int64_t tot = h.ngrid * PG * PG * PG;
  hipLaunchKernelGGL(hspec_kernel<T>, dim3((int)std::min<int64_t>((tot + kBlock - 1) / kBlock, 8192)), dim3(kBlock),
                     0, s, h);
  a.dcube = P.d_dcube;
  a.nspec = P.d_nspec;
  a.sbar = P.d_sbar;
  a.tab = P.d_cw2_tab;
  a.iw = P.d_axis_tab;
  a.modes = P.d_shell_modes;
  a.start = P.d_shell_start;
  a.combos = P.d_sn_combos;
  a.RF = P.RF;
  a.RG = P.RG;
  a.nb = P.nb;
  a.interlace = P.interlace;
  ylm_norm_table(a.ynorm);
  a.out = P.d_ssums;
  // (the 3PCF's r-bins have no shell sums: their kernel averages vanish)
  if (!P.sn_combos.empty() && !P.d_kslot)
    hipLaunchKernelGGL(shell_sums_kernel<T>, dim3((unsigned)P.sn_combos.size(), (unsigned)P.nb), dim3(kBlock), 0, s,
                       a);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

template <typename T>
int twopoint_impl(Plan& P, hipStream_t s) {
  const int nv = (int)P.sn_vlm.size();
  if (P.sn_zero_bin < 0 || nv == 0 || P.sn_combos.empty()) return TSB_OK;
  if (nv > kMaxV) return fail(TSB_E_UNSUPPORTED, "3PCF shot noise: too many two-point spectra");
  VArgs v{};
  v.dcube = P.d_dcube;
  v.nspec = P.d_nspec;
  v.vspec = P.d_vspec;
  v.sbar = P.d_sbar;
  v.tab = P.d_cw2_tab;
  v.iw = P.d_axis_tab;
  v.RF = P.RF;
  v.RG = P.RG;
  v.nv = nv;
  v.interlace = P.interlace;
  LMSrc src[81];
  int sre[81], sim[81];
  lm_sources(P, src, sre, sim);
  for (int k = 0; k < nv; ++k) {
    const int L = P.sn_vlm[k].L, M = P.sn_vlm[k].M, aM = M < 0 ? -M : M;
    v.src[k] = src[L * (L + 1) + M];
    v.sre[k] = (short)sre[L * (L + 1) + aM];
    v.sim[k] = (short)sim[L * (L + 1) + aM];
    v.sgn[k] = (short)(M < 0 ? ((aM & 1) ? -1 : 1) : 0);
  }
  const int64_t pf3 = (int64_t)P.PF * P.PF * P.PF;
  hipLaunchKernelGGL(vspec_kernel<T>, dim3((int)std::min<int64_t>((nv * pf3 + kBlock - 1) / kBlock, 8192)),
                     dim3(kBlock), 0, s, v);
  TSB_HIP(hipGetLastError());
  int rc;
  if ((rc = run_inverse_cube(P, P.d_vspec, nv, P.d_vfields, s))) return rc;
  TwoArgs t{};
  t.vfields = P.d_vfields;
  t.sep = P.d_shell_modes;
  t.start = P.d_shell_start;
  t.combos = P.d_sn_combos;
  t.N = P.N;
  t.RF = P.RF;
  t.nb = P.nb;
  ylm_norm_table(t.ynorm);
  t.out = P.d_ssums;
  hipLaunchKernelGGL(twopoint_sums_kernel<T>, dim3((unsigned)P.sn_combos.size(), (unsigned)P.nb), dim3(kBlock), 0, s,
                     t, (const int*)P.d_sn_combo_v);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

double alias_a(int p, double x) {
  const double s2 = std::sin(x) * std::sin(x);
  if (p == 1) return 1.0;
  if (p == 2) return 1.0 - 2.0 / 3.0 * s2;
  return 1.0 - s2 + 2.0 / 15.0 * s2 * s2;
}

double alias_b(int p, double x) {
  const double c = std::cos(x);
  if (p == 1) return c;
  if (p == 2) return (c * c * c + 5.0 * c) / 6.0;
  return (std::pow(c, 5) + 58.0 * c * c * c + 61.0 * c) / 120.0;
}

}  // namespace

int run_shot_kspace(Plan& P, hipStream_t s) {
  return P.precision == TSB_FP64 ? kspace_impl<double>(P, s) : kspace_impl<float>(P, s);
}

int run_separation_shot(Plan& P, hipStream_t s) {
  int rc = P.precision == TSB_FP64 ? separation_shot_impl<double>(P, s) : separation_shot_impl<float>(P, s);
  if (rc) return rc;
  return P.precision == TSB_FP64 ? twopoint_impl<double>(P, s) : twopoint_impl<float>(P, s);
}

// Host tables of a shot-noise plan: the complex terms of eq. 45 with the
// (l, m, L, M) shell sums they need, the lattice shell averages ybar, the shell
// mode list and the per-axis alias sums.
int shot_plan(Plan& P) {
  P.sn_terms.clear();
  P.sn_combos.clear();
  std::map<std::tuple<int, int, int, int>, int> cidx;
  auto combo = [&](int l, int m, int L, int M) {
    if (P.los_kind == TSB_LOS_GLOBAL) L = M = 0;   // N_L^M = y_L^M(d) N_0^0 (the factor is applied on the host)
    const auto key = std::make_tuple(l, m, L, M);
    auto it = cidx.find(key);
    if (it != cidx.end()) return it->second;
    const int k = (int)P.sn_combos.size();
    P.sn_combos.push_back({l, m, L, M});
    cidx[key] = k;
    return k;
  };
  for (int mu = 0; mu < (int)P.mult.size(); ++mu) {
    const int l1 = P.mult[mu].l1, l2 = P.mult[mu].l2, L = P.mult[mu].L;
    for (int m1 = -l1; m1 <= l1; ++m1)
      for (int m2 = -l2; m2 <= l2; ++m2) {
        const int M = -m1 - m2;
        if (std::abs(M) > L) continue;
        const double w = three_j(l1, l2, L, m1, m2, M);
        if (w == 0.0) continue;
        P.sn_terms.push_back({mu, m1, m2, M, w, combo(l1, m1, L, M), combo(l2, m2, L, M)});
      }
  }
  // lattice shell averages ybar_l^m*(b) for every l of the multipoles, all m.
  // The 3PCF's r-bins (none holds r = 0) have separation-kernel averages
  // (1/V) sum_k K = 0, which zero the other three terms: only the i = j != k
  // term remains, a sum over each bin's separation vectors (the list below).
  double norm[64];
  ylm_norm_table(norm);
  P.sn_ybar.assign((size_t)(kMaxEll + 1) * (kMaxEll + 1) * P.nb * 2, 0.0);
  std::vector<int> need(kMaxEll + 1, 0);
  for (auto& mp : P.mult) need[mp.l1] = need[mp.l2] = 1;
  const int RF = P.RF, PF = P.PF;
  std::vector<std::vector<int>> modes(P.nb);
  const bool xi = P.estimator != TSB_BISPECTRUM;
  for (int x = -RF; x <= RF; ++x)
    for (int y = -RF; y <= RF; ++y)
      for (int z = -RF; z <= RF; ++z) {
        const int64_t n2 = (int64_t)x * x + (int64_t)y * y + (int64_t)z * z;
        if ((n2 == 0 && !xi) || n2 > P.n2maxF) continue;   // (the zero separation is in its r-bin's list)
        const int b = P.bin_lut[n2];
        if (b < 0) continue;
        modes[b].push_back(((x + RF) * PF + (y + RF)) * PF + (z + RF));
        if (xi) continue;
        const double r = std::sqrt((double)n2), d[3] = {x / r, y / r, z / r};
        for (int l = 0; l <= kMaxEll; ++l) {
          if (!need[l]) continue;
          for (int m = -l; m <= l; ++m) {
            const std::complex<double> yc = std::conj(ylm_any(l, m, d, norm));
            const size_t k = ((size_t)(l * (l + 1) + m) * P.nb + b) * 2;
            P.sn_ybar[k] += yc.real();
            P.sn_ybar[k + 1] += yc.imag();
          }
        }
      }
  for (int l = 0; l <= kMaxEll; ++l)
    for (int m = -l; m <= l; ++m)
      for (int b = 0; b < P.nb; ++b) {
        const size_t k = ((size_t)(l * (l + 1) + m) * P.nb + b) * 2;
        if (P.nmode[b]) {
          P.sn_ybar[k] /= (double)P.nmode[b];
          P.sn_ybar[k + 1] /= (double)P.nmode[b];
        }
      }
  // shell mode list, or for the 3PCF the separation vectors of each r-bin
  // (device table built by the caller from these vectors)
  P.sn_mode_list.clear();
  P.sn_mode_start.assign(P.nb + 1, 0);
  for (int b = 0; b < P.nb; ++b) {
    P.sn_mode_start[b] = (int)P.sn_mode_list.size();
    P.sn_mode_list.insert(P.sn_mode_list.end(), modes[b].begin(), modes[b].end());
  }
  P.sn_mode_start[P.nb] = (int)P.sn_mode_list.size();
  // 3PCF: an r-bin holding the zero separation has the kernel average
  // Kbar_0^0 = N^3/(V N_r); the j = k and i = k terms then need the two-point
  // sums of every combo, from the inverse transforms of its (L, M) spectrum
  P.sn_zero_bin = -1;
  P.sn_vlm.clear();
  P.sn_combo_v.clear();
  if (xi && !P.bin_lut.empty() && P.bin_lut[0] >= 0) {
    P.sn_zero_bin = P.bin_lut[0];
    for (const Plan::SnCombo& c : P.sn_combos) {
      int v = -1;
      for (size_t k = 0; k < P.sn_vlm.size(); ++k)
        if (P.sn_vlm[k].L == c.L && P.sn_vlm[k].M == c.M) v = (int)k;
      if (v < 0) {
        v = (int)P.sn_vlm.size();
        P.sn_vlm.push_back({0, 0, c.L, c.M});
      }
      P.sn_combo_v.push_back(v);
    }
  }
  // alias sums per stored G-cube axis entry, x = pi n / N
  P.sn_alias.assign(2 * (size_t)P.PG, 0.0);
  for (int j = 0; j < P.PG; ++j) {
    const double x = M_PI * (double)(j - P.RG) / (double)P.N;
    P.sn_alias[j] = alias_a(P.p, x);
    P.sn_alias[P.PG + j] = alias_b(P.p, x);
  }
  return TSB_OK;
}

// After a measurement: the four terms of eq. 45 for every output, S, and
// B_out = B - S in the caller's layout (NaN where no pair is computed).
void shot_finish(Plan& P, const double* sbar, const double* sums, const double* Braw, const double* Sij, double I,
                 double* B_out) {
  typedef std::complex<double> cd;
  double norm[64];
  ylm_norm_table(norm);
  const size_t nbb = (size_t)P.nb * P.nb;
  const double nan = std::numeric_limits<double>::quiet_NaN();
  P.last_S.assign(P.mult.size() * nbb, nan);
  P.last_Sij.assign(P.mult.size() * nbb, nan);
  for (size_t i = 0; i < P.mult.size() * nbb; ++i) B_out[i] = nan;
  // Sbar_L^M (complex) from the real channels; a global LOS scales Sbar_0^0
  auto sbar_lm = [&](int L, int M) -> cd {
    if (P.los_kind == TSB_LOS_GLOBAL) return std::conj(ylm_any(L, M, P.los_dir, norm)) * cd(sbar[0], 0.0);
    const int aM = std::abs(M);
    double re = 0.0, im = 0.0;
    for (size_t c = 0; c < P.chans.size(); ++c) {
      if (P.chans[c].L != L || P.chans[c].M != aM) continue;
      (P.chans[c].part ? im : re) = sbar[c];
    }
    cd v(re, im);
    if (M < 0) v = ((aM & 1) ? -1.0 : 1.0) * std::conj(v);
    return v;
  };
  // The 3PCF (reading of eq. 51): the kernel averages (1/V) sum_k K vanish but
  // for the zero separation's bin, where Kbar_0^0 = N^3 / (V N_r); the
  // two-point sums carry 1/(V N_r) instead of the shell average's 1/N_mode.
  const bool xi = P.estimator != TSB_BISPECTRUM;
  const double V = P.L * P.L * P.L, N3 = (double)P.N * P.N * P.N;
  auto ybar = [&](int l, int m, int b) {
    if (xi) return cd(b == P.sn_zero_bin && l == 0 && m == 0 ? N3 / (V * (double)P.nmode[b]) : 0.0, 0.0);
    const size_t k = ((size_t)(l * (l + 1) + m) * P.nb + b) * 2;
    return cd(P.sn_ybar[k], P.sn_ybar[k + 1]);
  };
  auto A = [&](int combo, int L, int M, int b) {
    cd v(sums[((size_t)combo * P.nb + b) * 2], sums[((size_t)combo * P.nb + b) * 2 + 1]);
    v /= (double)P.nmode[b] * (xi ? V : 1.0);
    if (P.los_kind == TSB_LOS_GLOBAL) v *= std::conj(ylm_any(L, M, P.los_dir, norm));
    return v;
  };
  for (size_t o = 0; o < P.outs.size(); ++o) {
    const OutEntry& e = P.outs[o];
    const int l1 = P.mult[e.mu].l1, l2 = P.mult[e.mu].l2, L = P.mult[e.mu].L;
    const double pref = P.mu_pref[e.mu] / I;
    cd t(0.0, 0.0);
    for (const Plan::SnTerm& st : P.sn_terms) {
      if (st.mu != e.mu || (xi && P.sn_zero_bin < 0)) continue;   // (3PCF without the zero bin: i = j != k only)
      const cd y1 = ybar(l1, st.m1, e.b1), y2 = ybar(l2, st.m2, e.b2);
      t += st.w3j * (y1 * y2 * sbar_lm(L, st.M) + A(st.cjk, L, st.M, e.b1) * y2 + y1 * A(st.cik, L, st.M, e.b2));
    }
    const double S = pref * t.real() + Sij[o];
    const size_t at = (size_t)e.mu * nbb + (size_t)e.b1 * P.nb + e.b2;
    P.last_S[at] = S;
    P.last_Sij[at] = Sij[o];
    B_out[at] = Braw[o] - S;
  }
}

}  // namespace tsb
