// Masked model of the three-point-function and bispectrum multipoles
// (Sec. 6.2): the window multipoles Q measured by the library couple the
// model multipoles zeta through Wigner 9j symbols (eq. 63, App. A), the
// integral constraint removes the survey-mean term (eq. 64), and a double
// spherical Hankel transform turns the masked zeta into the masked bispectrum
// (eq. 68). Host code: the inputs are a few hundred r-bin pairs per multipole.
//
// The 9j symbol is the sum over x of three 6j symbols (the standard
// recoupling sum), the 6j is Racah's formula in long double; the spherical
// Bessel functions use the power series for small arguments, Miller's
// downward recurrence normalised by j_0 below the order and the upward
// recurrence above it. The r integrals are quadrature sums with the caller's
// weights.
#include <cmath>
#include <vector>

#include "tsb_internal.h"

namespace tsb {

namespace {

constexpr int kMaxMaskEll = 16;

long double fact(int n) {
  static long double tab[4 * kMaxMaskEll + 8];
  static bool init = false;
  if (!init) {
    tab[0] = 1.0L;
    for (int i = 1; i < 4 * kMaxMaskEll + 8; ++i) tab[i] = tab[i - 1] * (long double)i;
    init = true;
  }
  return tab[n];
}

bool triad(int a, int b, int c) { return c >= std::abs(a - b) && c <= a + b; }

long double delta(int a, int b, int c) {
  return std::sqrt(fact(a + b - c) * fact(a - b + c) * fact(-a + b + c) / fact(a + b + c + 1));
}

// {j1 j2 j3; j4 j5 j6}, Racah's formula
long double six_j(int j1, int j2, int j3, int j4, int j5, int j6) {
  if (!triad(j1, j2, j3) || !triad(j1, j5, j6) || !triad(j4, j2, j6) || !triad(j4, j5, j3)) return 0.0L;
  const int a1 = j1 + j2 + j3, a2 = j1 + j5 + j6, a3 = j4 + j2 + j6, a4 = j4 + j5 + j3;
  const int b1 = j1 + j2 + j4 + j5, b2 = j2 + j3 + j5 + j6, b3 = j3 + j1 + j6 + j4;
  const int tmin = std::max({a1, a2, a3, a4}), tmax = std::min({b1, b2, b3});
  long double s = 0.0L;
  for (int t = tmin; t <= tmax; ++t) {
    const long double term = fact(t + 1) / (fact(t - a1) * fact(t - a2) * fact(t - a3) * fact(t - a4) *
                                            fact(b1 - t) * fact(b2 - t) * fact(b3 - t));
    s += (t % 2) ? -term : term;
  }
  return delta(j1, j2, j3) * delta(j1, j5, j6) * delta(j4, j2, j6) * delta(j4, j5, j3) * s;
}

// {a b c; d e f; g h i} = sum_x (2x+1) {a b c; f i x} {d e f; b x h} {g h i; x a d}
// (integer arguments, so (-1)^{2x} = 1)
double nine_j(int a, int b, int c, int d, int e, int f, int g, int h, int i) {
  const int xmin = std::max({std::abs(a - i), std::abs(d - h), std::abs(b - f)});
  const int xmax = std::min({a + i, d + h, b + f});
  long double s = 0.0L;
  for (int x = xmin; x <= xmax; ++x)
    s += (long double)(2 * x + 1) * six_j(a, b, c, f, i, x) * six_j(d, e, f, b, x, h) * six_j(g, h, i, x, a, d);
  return (double)s;
}

// j_l(x), x >= 0
double sph_bessel(int l, double x) {
  if (x == 0.0) return l == 0 ? 1.0 : 0.0;
  if (x < 0.5) {
    // x^l / (2l+1)!! * sum_k (-x^2/2)^k / (k! (2l+3)(2l+5)...(2l+2k+1))
    double pre = 1.0;
    for (int n = 1; n <= l; ++n) pre *= x / (double)(2 * n + 1);
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 30; ++k) {
      term *= -0.5 * x * x / ((double)k * (double)(2 * l + 2 * k + 1));
      sum += term;
      if (std::fabs(term) < 1e-18 * std::fabs(sum)) break;
    }
    return pre * sum;
  }
  const double j0 = std::sin(x) / x;
  if (l == 0) return j0;
  if (x > (double)l) {
    double jm = j0, jc = std::sin(x) / (x * x) - std::cos(x) / x;
    for (int n = 1; n < l; ++n) {
      const double jn = (2.0 * n + 1.0) / x * jc - jm;
      jm = jc;
      jc = jn;
    }
    return jc;
  }
  // Miller: downward from well above l, normalised by j_0
  const int nstart = l + 30 + (int)x;
  double jp = 0.0, jc = 1e-300, want = 0.0;
  for (int n = nstart; n >= 1; --n) {
    const double jn = (2.0 * n + 1.0) / x * jc - jp;
    jp = jc;
    jc = jn;
    if (n - 1 == l) want = jc;
    if (std::fabs(jc) > 1e250) {   // rescale
      jc *= 1e-250;
      jp *= 1e-250;
      want *= 1e-250;
    }
  }
  return want * (j0 / jc);
}

bool multipole_ok(const tsb_multipole& m) {
  return m.l1 >= 0 && m.l2 >= 0 && m.L >= 0 && m.l1 <= kMaxMaskEll && m.l2 <= kMaxMaskEll && m.L <= kMaxMaskEll;
}

double hfac(int a, int b, int c) { return three_j(a, b, c, 0, 0, 0); }
double nfac(int a, int b, int c) { return (double)((2 * a + 1) * (2 * b + 1) * (2 * c + 1)); }

}  // namespace

}  // namespace tsb

using namespace tsb;

extern "C" {

int tsb_wigner_9j(const int32_t* l, double* out) {
  if (!l || !out) return fail(TSB_E_ARG, "NULL argument");
  for (int i = 0; i < 9; ++i)
    if (l[i] < 0 || l[i] > kMaxMaskEll) return fail(TSB_E_UNSUPPORTED, "9j arguments must be in 0..16");
  *out = nine_j(l[0], l[1], l[2], l[3], l[4], l[5], l[6], l[7], l[8]);
  return TSB_OK;
}

int tsb_masked_zeta(const tsb_multipole* model, int32_t n_model, const double* zeta, const tsb_multipole* window,
                    int32_t n_window, const double* Q, const double* r, const double* w, int32_t n_r,
                    const tsb_multipole* out, int32_t n_out, int32_t integral_constraint, double* zeta_out,
                    double* zeta_bar) {
  if (!model || !zeta || !window || !Q || !out || !zeta_out) return fail(TSB_E_ARG, "NULL argument");
  if (n_model < 1 || n_window < 1 || n_out < 1 || n_r < 1) return fail(TSB_E_ARG, "empty multipole set or r grid");
  if (integral_constraint && (!r || !w)) return fail(TSB_E_ARG, "the integral constraint needs r and its weights");
  for (int i = 0; i < n_model; ++i)
    if (!multipole_ok(model[i])) return fail(TSB_E_UNSUPPORTED, "model multipole l outside 0..16");
  for (int i = 0; i < n_window; ++i)
    if (!multipole_ok(window[i])) return fail(TSB_E_UNSUPPORTED, "window multipole l outside 0..16");
  for (int i = 0; i < n_out; ++i)
    if (!multipole_ok(out[i])) return fail(TSB_E_UNSUPPORTED, "output multipole l outside 0..16");
  const int64_t nn = (int64_t)n_r * n_r;
  auto same = [](const tsb_multipole& a, const tsb_multipole& b) { return a.l1 == b.l1 && a.l2 == b.l2 && a.L == b.L; };
  // integral constraint (eq. 64): sum over multipoles in both sets of
  // int r1^2 r2^2 Q zeta / (H^2 N), over int r1^2 r2^2 Q_000
  double zbar = 0.0;
  if (integral_constraint) {
    int q0 = -1;
    for (int j = 0; j < n_window; ++j)
      if (window[j].l1 == 0 && window[j].l2 == 0 && window[j].L == 0) q0 = j;
    if (q0 < 0) return fail(TSB_E_ARG, "the integral constraint needs Q_000 among the window multipoles");
    std::vector<double> q(n_r);
    for (int i = 0; i < n_r; ++i) q[i] = w[i] * r[i] * r[i];
    auto integral = [&](const double* a, const double* b) {
      long double s = 0.0L;
      for (int i = 0; i < n_r; ++i)
        for (int j = 0; j < n_r; ++j) {
          const int64_t e = (int64_t)i * n_r + j;
          s += (long double)q[i] * q[j] * a[e] * (b ? b[e] : 1.0);
        }
      return (double)s;
    };
    const double den = integral(Q + (int64_t)q0 * nn, nullptr);
    if (!(den != 0.0) || !std::isfinite(den)) return fail(TSB_E_INPUT, "the r1^2 r2^2 integral of Q_000 is zero");
    double num = 0.0;
    for (int a = 0; a < n_model; ++a)
      for (int b = 0; b < n_window; ++b) {
        if (!same(model[a], window[b])) continue;
        const double h = hfac(model[a].l1, model[a].l2, model[a].L);
        if (h == 0.0) continue;
        num += integral(Q + (int64_t)b * nn, zeta + (int64_t)a * nn) / (h * h * nfac(model[a].l1, model[a].l2, model[a].L));
      }
    zbar = num / den;
  }
  if (zeta_bar) *zeta_bar = zbar;
  // eq. 63
  for (int o = 0; o < n_out; ++o) {
    const int l1 = out[o].l1, l2 = out[o].l2, L = out[o].L;
    double* dst = zeta_out + (int64_t)o * nn;
    for (int64_t e = 0; e < nn; ++e) dst[e] = 0.0;
    const double hout = hfac(l1, l2, L);
    for (int a = 0; a < n_model; ++a) {
      const int a1 = model[a].l1, a2 = model[a].l2, aL = model[a].L;
      const double ha = hfac(a1, a2, aL);
      for (int b = 0; b < n_window; ++b) {
        const int b1 = window[b].l1, b2 = window[b].l2, bL = window[b].L;
        const double hb = hfac(b1, b2, bL);
        if (ha == 0.0 || hb == 0.0) continue;
        const double num = hout * hfac(l1, a1, b1) * hfac(l2, a2, b2) * hfac(L, aL, bL);
        if (num == 0.0) continue;
        const double c = nfac(l1, l2, L) * nine_j(b1, b2, bL, a1, a2, aL, l1, l2, L) * num / (ha * hb);
        if (c == 0.0) continue;
        const double* qa = Q + (int64_t)b * nn;
        const double* za = zeta + (int64_t)a * nn;
        for (int64_t e = 0; e < nn; ++e) dst[e] += c * qa[e] * za[e];
      }
    }
    if (integral_constraint)
      for (int b = 0; b < n_window; ++b)
        if (same(window[b], out[o])) {
          const double* qa = Q + (int64_t)b * nn;
          for (int64_t e = 0; e < nn; ++e) dst[e] -= qa[e] * zbar;
        }
  }
  return TSB_OK;
}

int tsb_masked_bispectrum(int32_t l1, int32_t l2, const double* zeta, const double* r, const double* w, int32_t n_r,
                          const double* k, int32_t n_k, double* B_out) {
  if (!zeta || !r || !w || !k || !B_out) return fail(TSB_E_ARG, "NULL argument");
  if (n_r < 1 || n_k < 1) return fail(TSB_E_ARG, "empty r or k grid");
  if (l1 < 0 || l2 < 0 || l1 > kMaxMaskEll || l2 > kMaxMaskEll) return fail(TSB_E_UNSUPPORTED, "l outside 0..16");
  if ((l1 + l2) % 2) return fail(TSB_E_UNSUPPORTED, "l1 + l2 must be even (a real transform)");
  for (int i = 0; i < n_r; ++i)
    if (!(r[i] >= 0.0)) return fail(TSB_E_ARG, "r must be >= 0");
  for (int i = 0; i < n_k; ++i)
    if (!(k[i] >= 0.0)) return fail(TSB_E_ARG, "k must be >= 0");
  // J_l[a][i] = w_i r_i^2 j_l(k_a r_i); B = (-i)^{l1+l2} (4 pi)^2 J_l1 zeta J_l2^T
  std::vector<double> J1((size_t)n_k * n_r), J2((size_t)n_k * n_r);
  for (int a = 0; a < n_k; ++a)
    for (int i = 0; i < n_r; ++i) {
      const double q = w[i] * r[i] * r[i];
      J1[(size_t)a * n_r + i] = q * sph_bessel(l1, k[a] * r[i]);
      J2[(size_t)a * n_r + i] = q * sph_bessel(l2, k[a] * r[i]);
    }
  const double pref = (((l1 + l2) / 2) % 2 ? -1.0 : 1.0) * 16.0 * M_PI * M_PI;
  std::vector<double> T((size_t)n_k * n_r);   // J1 zeta
  for (int a = 0; a < n_k; ++a)
    for (int j = 0; j < n_r; ++j) {
      long double s = 0.0L;
      for (int i = 0; i < n_r; ++i) s += (long double)J1[(size_t)a * n_r + i] * zeta[(size_t)i * n_r + j];
      T[(size_t)a * n_r + j] = (double)s;
    }
  for (int a = 0; a < n_k; ++a)
    for (int b = 0; b < n_k; ++b) {
      long double s = 0.0L;
      for (int j = 0; j < n_r; ++j) s += (long double)T[(size_t)a * n_r + j] * J2[(size_t)b * n_r + j];
      B_out[(size_t)a * n_k + b] = pref * (double)s;
    }
  return TSB_OK;
}

}  // extern "C"
