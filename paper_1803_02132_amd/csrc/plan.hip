// Host-side planning: validation, k-shells, the reduction grid, channel and
// slot layout, and the real expansion of the 3j-weighted m-sum of eq. 41.
#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <tuple>

#include "tsb_internal.h"

namespace tsb {

namespace {

typedef std::complex<double> cd;

long double lfact(int n) {
  long double r = 1.0L;
  for (int i = 2; i <= n; ++i) r *= (long double)i;
  return r;
}

}  // namespace

// Wigner 3j symbol by Racah's formula in extended precision (Sec. 2, eq. 11).
double three_j(int j1, int j2, int j3, int m1, int m2, int m3) {
  if (m1 + m2 + m3 != 0) return 0.0;
  if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(m3) > j3) return 0.0;
  if (j3 < std::abs(j1 - j2) || j3 > j1 + j2) return 0.0;
  int kmin = std::max({0, j2 - j3 - m1, j1 - j3 + m2});
  int kmax = std::min({j1 + j2 - j3, j1 - m1, j2 + m2});
  long double s = 0.0L;
  for (int k = kmin; k <= kmax; ++k) {
    long double den = lfact(k) * lfact(j3 - j2 + k + m1) * lfact(j3 - j1 + k - m2) *
                      lfact(j1 + j2 - j3 - k) * lfact(j1 - k - m1) * lfact(j2 - k + m2);
    s += ((k % 2) ? -1.0L : 1.0L) / den;
  }
  long double tri = lfact(j1 + j2 - j3) * lfact(j1 - j2 + j3) * lfact(-j1 + j2 + j3) /
                    lfact(j1 + j2 + j3 + 1);
  long double f = lfact(j1 + m1) * lfact(j1 - m1) * lfact(j2 + m2) * lfact(j2 - m2) *
                  lfact(j3 + m3) * lfact(j3 - m3);
  long double v = std::sqrt(tri * f) * s;
  int ph = j1 - j2 - m3;
  if (((ph % 2) + 2) % 2) v = -v;
  return (double)v;
}

namespace {

bool is_2a3b(int n) {
  if (n <= 0) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

}  // namespace

// y_L^M(d) for any M via y^{-M} = (-1)^M conj(y^M), with the device routine.
std::complex<double> ylm_any(int l, int m, const double* d, const double* norm) {
  double re, im;
  ylm_pos_m(l, std::abs(m), d[0], d[1], d[2], norm, &re, &im);
  cd v(re, im);
  if (m < 0) v = ((std::abs(m) % 2) ? -1.0 : 1.0) * std::conj(v);
  return v;
}

void ylm_norm_table(double* norm) {
  for (int l = 0; l <= kMaxEll; ++l)
    for (int m = 0; m <= l; ++m) {
      long double r = std::sqrt(lfact(l - m) / lfact(l + m));
      norm[l * (l + 1) / 2 + m] = (double)((m % 2) ? -r : r);
    }
}

// Whether an unfused FP32 plan reduces on the matrix cores in the kernel with
// its terms in the kernel arguments (at most 32 shells, 16 Q groups, 64 terms).
bool unfused_mfma_applies(const Plan& P) {
  return P.precision == TSB_FP32 && P.nb <= 32 && P.red_chunk % 8 == 0 && P.fkinds.size() <= 32 &&
         P.grids.size() <= 32 && P.qgroups.size() >= 1 && P.qgroups.size() <= 16 && P.terms.size() <= 64;
}

int plan_build(Plan& P) {
  const int N = P.N;
  if (N < 16 || N > 1024 || N % 4 != 0 || !is_2a3b(N))
    return fail(TSB_E_UNSUPPORTED, "grid size N must be 2^a 3^b with 16 <= N <= 1024 and N % 4 == 0");
  if (!(P.L > 0) || !std::isfinite(P.L)) return fail(TSB_E_ARG, "box_len must be positive");
  if (P.p < 1 || P.p > 3) return fail(TSB_E_ARG, "assign_p must be 1 (NGP), 2 (CIC) or 3 (TSC)");
  if (P.interlace != 0 && P.interlace != 1) return fail(TSB_E_ARG, "interlace must be 0 or 1");
  if (P.nb < 1 || P.nb > kMaxBins) return fail(TSB_E_ARG, "n_bins must be in 1..64");
  if (P.edges.empty()) {
    if (!(P.dk > 0) || !(P.kmin >= 0) || !std::isfinite(P.dk) || !std::isfinite(P.kmin))
      return fail(TSB_E_ARG, "need dk > 0 and k_min >= 0");
  } else {
    if ((int)P.edges.size() != P.nb + 1) return fail(TSB_E_ARG, "edges must hold n_bins + 1 values");
    for (int b = 0; b <= P.nb; ++b)
      if (!std::isfinite(P.edges[b]) || P.edges[b] < 0 || (b > 0 && !(P.edges[b] > P.edges[b - 1])))
        return fail(TSB_E_ARG, "edges must be finite, >= 0 and strictly increasing");
  }
  if (P.vertex != TSB_VERTEX_X3 && P.vertex != TSB_VERTEX_X1 && P.vertex != TSB_VERTEX_X2)
    return fail(TSB_E_ARG, "los vertex must be 0 (x3), 1 (x1) or 2 (x2)");
  if (P.estimator < TSB_BISPECTRUM || P.estimator > TSB_WINDOW) return fail(TSB_E_ARG, "estimator must be 0, 1 or 2");
  if (P.shot_noise != 0 && P.shot_noise != 1) return fail(TSB_E_ARG, "shot_noise must be 0 or 1");
  // LOS at the first or second vertex (App. B): the y_L^M* weight moves from G
  // onto that shell field; under a global LOS every vertex is the same estimator
  const bool x1 = P.vertex == TSB_VERTEX_X1 && P.los_kind == TSB_LOS_LOCAL;
  const bool x2 = P.vertex == TSB_VERTEX_X2 && P.los_kind == TSB_LOS_LOCAL;
  P.g00_only = x1 || x2;
  if (P.g00_only && P.estimator != TSB_BISPECTRUM)
    return fail(TSB_E_UNSUPPORTED, "the first- and second-vertex LOS are built for the bispectrum");
  if (P.g00_only && P.shot_noise) return fail(TSB_E_UNSUPPORTED, "the shot noise is built for the third-vertex LOS");
  const bool xi = P.estimator != TSB_BISPECTRUM;   // separation bins (Sec. 4.3, 6.1)
  if (P.estimator == TSB_WINDOW && P.shot_noise)
    return fail(TSB_E_UNSUPPORTED, "shot-noise subtraction is for the bispectrum and the 3PCF");
  if (P.estimator == TSB_WINDOW && P.box_mode)
    return fail(TSB_E_UNSUPPORTED, "window multipoles need a random catalogue (survey mode)");
  if (P.mult.empty()) return fail(TSB_E_ARG, "no multipoles");
  if (P.los_kind != TSB_LOS_GLOBAL && P.los_kind != TSB_LOS_LOCAL)
    return fail(TSB_E_ARG, "los kind must be global (0) or local (1)");
  if (P.precision != TSB_FP32 && P.precision != TSB_FP64) return fail(TSB_E_ARG, "precision");
  if (P.pair_mode < 0 || P.pair_mode > 3) return fail(TSB_E_ARG, "pair_mode");
  for (auto& mp : P.mult) {
    int l1 = mp.l1, l2 = mp.l2, L = mp.L;
    if (l1 < 0 || l2 < 0 || L < 0 || l1 > kMaxEll || l2 > kMaxEll || L > kMaxEll)
      return fail(TSB_E_UNSUPPORTED, "l1, l2, L must be in 0..8");
    // Table 1 (Sec. 2): L even, triangle rule, l1 + l2 + L even
    if (L % 2 || L < std::abs(l1 - l2) || L > l1 + l2 || (l1 + l2 + L) % 2)
      return fail(TSB_E_UNSUPPORTED, "multipole outside the allowed set of Table 1");
  }
  if (P.los_kind == TSB_LOS_GLOBAL) {
    double n2 = P.los_dir[0] * P.los_dir[0] + P.los_dir[1] * P.los_dir[1] + P.los_dir[2] * P.los_dir[2];
    if (!(n2 > 0)) return fail(TSB_E_ARG, "global LOS direction is zero");
    double s = 1.0 / std::sqrt(n2);
    for (int a = 0; a < 3; ++a) P.los_dir[a] *= s;
  }
  P.copies = 1 + P.interlace;

  // ---- k-shells (eq. 38), or separation bins of the 3PCF: bin of every
  // integer n^2 (|k| = k_f sqrt(n^2); |r| = H sqrt(n^2), n = 0 included) ------
  const double kf = 2.0 * M_PI / P.L;
  const double unit = xi ? P.L / N : kf;
  const int64_t h = N / 2;
  const int64_t n2all = 3 * h * h;
  std::vector<int> lut(n2all + 1, -1);
  int64_t n2maxF = 0;
  for (int64_t n2 = xi ? 0 : 1; n2 <= n2all; ++n2) {
    const double k = unit * std::sqrt((double)n2);
    int bin = -1;
    if (P.edges.empty()) {
      const double b = std::floor((k - P.kmin) / P.dk);
      if (b >= 0 && b < P.nb) bin = (int)b;
    } else if (k >= P.edges[0] && k < P.edges[P.nb]) {
      // [edges[b], edges[b+1]): the last edge not above k
      bin = (int)(std::upper_bound(P.edges.begin(), P.edges.end(), k) - P.edges.begin()) - 1;
    }
    if (bin >= 0) {
      lut[n2] = bin;
      n2maxF = n2;
    }
  }
  bool any_bin = false;
  for (int64_t n2 = 0; n2 <= n2all; ++n2) any_bin = any_bin || lut[n2] >= 0;
  if (!any_bin) return fail(TSB_E_UNSUPPORTED, xi ? "no grid separation falls in any r-bin"
                                                  : "no grid mode falls in any k-shell");
  // no shell may hold a mode with an index component of N/2 (those are zeroed);
  // r-bins stay inside half the box (r and -r distinct)
  for (int64_t n2 = h * h; n2 <= n2all; ++n2)
    if (lut[n2] >= 0)
      return fail(TSB_E_UNSUPPORTED, xi ? "r-bins reach half the box" : "k-shells reach the Nyquist frequency");
  int RF;
  if (xi) {
    // the 3PCF filters every mode: F and G cover the whole (non-Nyquist) cube
    RF = (int)h - 1;
    P.n2maxF = 3 * (int64_t)RF * RF;
  } else {
    P.n2maxF = n2maxF;
    RF = (int)std::floor(std::sqrt((double)n2maxF));
    while ((int64_t)(RF + 1) * (RF + 1) <= n2maxF) ++RF;
    while ((int64_t)RF * RF > n2maxF) --RF;
  }
  P.RF = RF;
  P.bin_lut.assign(lut.begin(), lut.begin() + (3 * (int64_t)RF * RF + 1));

  // ---- reduction grid ---------------------------------------------------------
  // With every shell inside |n| <= sqrt(n2maxF), F1 F2 only meets G at modes with
  // |n3| <= 2 sqrt(n2maxF). If 2 RF < N/2 no F pair wraps on the N grid, and the
  // sum over cells of F F G equals (N/M)^3 times the same sum on any M grid with
  // M > 2 RF + RG: then no closed triangle aliases onto another.
  if (!xi && 4 * RF < N) {
    P.n2maxG = 4 * n2maxF;
    int RG = (int)std::floor(2.0 * std::sqrt((double)n2maxF));
    while ((int64_t)(RG + 1) * (RG + 1) <= P.n2maxG) ++RG;
    while ((int64_t)RG * RG > P.n2maxG) --RG;
    RG = std::min(RG, N / 2 - 1);
    P.RG = RG;
    int mmin = 2 * RF + RG + 1;
    int M = N;
    for (int a = 4; a <= N; a *= 2)
      for (int b = a; b <= N; b *= 3)
        if (b >= mmin && b < M && b % 4 == 0) M = b;
    P.M = M;
  } else {
    P.n2maxG = -1;
    P.RG = N / 2 - 1;
    P.M = N;
  }
  P.PF = 2 * P.RF + 1;
  P.PG = 2 * P.RG + 1;

  // N_mode and mean |k| per shell (all modes of a shell are in the F cube)
  P.nmode.assign(P.nb, 0);
  P.keff.assign(P.nb, 0.0);
  // (3PCF: N_r and the mean |r| of the separation vectors of each bin)
  for (int x = -RF; x <= RF; ++x)
    for (int y = -RF; y <= RF; ++y)
      for (int z = -RF; z <= RF; ++z) {
        int64_t n2 = (int64_t)x * x + (int64_t)y * y + (int64_t)z * z;
        if (n2 > P.n2maxF) continue;
        int b = P.bin_lut[n2];
        if (b < 0) continue;
        P.nmode[b] += 1;
        P.keff[b] += unit * std::sqrt((double)n2);
      }
  for (int b = 0; b < P.nb; ++b) P.keff[b] = P.nmode[b] ? P.keff[b] / P.nmode[b] : NAN;

  // ---- channels and complex grids ------------------------------------------------
  std::vector<int> Ls{0};
  if (P.los_kind == TSB_LOS_LOCAL)
    for (auto& mp : P.mult)
      if (std::find(Ls.begin(), Ls.end(), mp.L) == Ls.end()) Ls.push_back(mp.L);
  std::sort(Ls.begin(), Ls.end());
  P.chans.clear();
  P.grids.clear();
  std::vector<int> m0;
  for (int L : Ls) {
    m0.push_back((int)P.chans.size());
    P.chans.push_back({L, 0, 0});
  }
  for (size_t i = 0; i < m0.size(); i += 2)
    P.grids.push_back({m0[i], i + 1 < m0.size() ? m0[i + 1] : -1});
  for (int L : Ls)
    for (int M = 1; M <= L; ++M) {
      int c = (int)P.chans.size();
      P.chans.push_back({L, M, 0});
      P.chans.push_back({L, M, 1});
      P.grids.push_back({c, c + 1});
    }
  // (L, M, part) -> G component (grid, part); the LOS at the first or second
  // vertex needs G_0^0 only (grid 0, real part), the other grids feed the
  // weighted shell fields
  std::map<std::tuple<int, int, int>, int> gkey;
  P.gcomp.clear();
  for (int g = 0; g < (int)P.grids.size(); ++g) {
    for (int part = 0; part < 2; ++part) {
      int c = part ? P.grids[g].im : P.grids[g].re;
      if (c < 0) continue;
      const RealChannel& ch = P.chans[c];
      if (P.g00_only && (ch.L != 0 || ch.M != 0)) continue;
      gkey[std::make_tuple(ch.L, ch.M, ch.part)] = (int)P.gcomp.size();
      P.gcomp.push_back({g, part});
    }
  }

  // ---- expansion of Re sum_{m1 m2 M} 3j F F G into real triple products --------
  double norm[64];
  ylm_norm_table(norm);
  // logical F components: (l, m, part, L, M) for the shell field of
  // y_l^m*(k^) dn_L^M(k); dn_0^0 (L = M = 0) for every field of the
  // third-vertex LOS and for the unweighted field of the first- or
  // second-vertex one. Of
  // each conjugate pair, F_{l L}^{-m -M} = (-1)^{l+m+M} conj(F_{l L}^{m M})
  // (real catalogue weights), the member with M > 0, or M = 0 and m >= 0, is
  // kept: part 0/1 = its Re/Im, or for m = M = 0 part 0 = the real field
  // c_l F (c_l = 1 for even l, -i for odd l).
  typedef std::tuple<int, int, int, int, int> LKey;
  std::map<std::tuple<int, LKey, LKey, int>, double> acc;   // (mu, f1, f2, g) -> coef
  auto ffactor = [](int l, int m, int L = 0, int M = 0) {
    std::vector<std::pair<LKey, cd>> out;
    const bool keep = M > 0 || (M == 0 && m >= 0);
    const int mc = keep ? m : -m, Mc = keep ? M : -M;
    if (mc == 0 && Mc == 0) {
      cd inv_c = (l % 2) ? cd(0, 1) : cd(1, 0);   // 1/c_l
      out.push_back({LKey(l, 0, 0, L, 0), inv_c});
    } else if (keep) {
      out.push_back({LKey(l, mc, 0, L, Mc), cd(1, 0)});
      out.push_back({LKey(l, mc, 1, L, Mc), cd(0, 1)});
    } else {
      double s = ((l + std::abs(m) + std::abs(M)) % 2) ? -1.0 : 1.0;
      out.push_back({LKey(l, mc, 0, L, Mc), cd(s, 0)});
      out.push_back({LKey(l, mc, 1, L, Mc), cd(0, -s)});
    }
    return out;
  };
  auto gfactor = [&](int L, int M) {
    std::vector<std::pair<int, cd>> out;
    if (P.g00_only) {   // the weight sits in the first or second field
      out.push_back({gkey.at(std::make_tuple(0, 0, 0)), cd(1, 0)});
      return out;
    }
    if (P.los_kind == TSB_LOS_GLOBAL) {
      // Sec. 4.4 with a general direction: G_L^M = y_L^M*(d) G_0^0
      cd y = std::conj(ylm_any(L, M, P.los_dir, norm));
      if (std::abs(y) > 1e-15) out.push_back({gkey.at(std::make_tuple(0, 0, 0)), y});
      return out;
    }
    int aM = std::abs(M);
    if (M == 0) {
      out.push_back({gkey.at(std::make_tuple(L, 0, 0)), cd(1, 0)});
    } else if (M > 0) {
      out.push_back({gkey.at(std::make_tuple(L, aM, 0)), cd(1, 0)});
      out.push_back({gkey.at(std::make_tuple(L, aM, 1)), cd(0, 1)});
    } else {
      double s = (aM % 2) ? -1.0 : 1.0;          // G^{-M} = (-1)^M conj(G^M)
      out.push_back({gkey.at(std::make_tuple(L, aM, 0)), cd(s, 0)});
      out.push_back({gkey.at(std::make_tuple(L, aM, 1)), cd(0, -s)});
    }
    return out;
  };
  // 3PCF: the F fields are built from the separation kernels K'_l^m = i^-l K_l^m
  // (K of eq. 49 on the grid), which have the parity of y_l^m*(k^) and so keep
  // the symmetries used below; F = i^l F', and the phase i^(l1+l2) moves into
  // the coefficients (the fields of every term are real)
  P.mu_pref.assign(P.mult.size(), 0.0);
  for (int mu = 0; mu < (int)P.mult.size(); ++mu) {
    int l1 = P.mult[mu].l1, l2 = P.mult[mu].l2, L = P.mult[mu].L;
    static const cd ipow[4] = {cd(1, 0), cd(0, 1), cd(-1, 0), cd(0, -1)};
    const cd phase = xi ? ipow[(l1 + l2) % 4] : cd(1, 0);
    P.mu_pref[mu] = (double)((2 * l1 + 1) * (2 * l2 + 1) * (2 * L + 1)) * three_j(l1, l2, L, 0, 0, 0);
    for (int m1 = -l1; m1 <= l1; ++m1)
      for (int m2 = -l2; m2 <= l2; ++m2) {
        int M = -m1 - m2;
        if (std::abs(M) > L) continue;
        double w = three_j(l1, l2, L, m1, m2, M);
        if (w == 0.0) continue;
        for (auto& a : (x1 ? ffactor(l1, m1, L, M) : ffactor(l1, m1)))
          for (auto& b : (x2 ? ffactor(l2, m2, L, M) : ffactor(l2, m2)))
            for (auto& c : gfactor(L, M)) {
              double re = (phase * w * a.second * b.second * c.second).real();
              acc[std::make_tuple(mu, a.first, b.first, c.first)] += re;
            }
      }
  }
  // keep the non-vanishing real terms and the F components they use
  std::map<LKey, int> used;
  std::vector<std::tuple<int, LKey, LKey, int, double>> kept;
  for (auto& kv : acc) {
    if (std::abs(kv.second) < 1e-13) continue;
    kept.push_back(std::make_tuple(std::get<0>(kv.first), std::get<1>(kv.first),
                                   std::get<2>(kv.first), std::get<3>(kv.first), kv.second));
    used[std::get<1>(kv.first)] = 1;
    used[std::get<2>(kv.first)] = 1;
  }
  // source of the shell filter of dn_L^M (M >= 0): dn_0^0 is the prepared F
  // cube; otherwise the spectrum of the complex grid that holds the channel,
  // itself for M > 0 (its grid is Re + i Im of dn_L^M), or the Hermitian part
  // of a packed pair of real M = 0 channels
  auto source = [&](FPart& fp, int L, int M) {
    fp.src = -1;
    fp.smode = 0;
    if (L == 0 && M == 0) return;
    for (int g = 0; g < (int)P.grids.size(); ++g)
      for (int part = 0; part < 2; ++part) {
        const int c = part ? P.grids[g].im : P.grids[g].re;
        if (c < 0 || P.chans[c].L != L || P.chans[c].M != M || P.chans[c].part != 0) continue;
        fp.src = g;
        fp.smode = M > 0 ? 0 : 1 + part;
      }
  };
  // F slot kinds: one complex slot per (l, m, L, M) kept with M > 0 or m > 0;
  // the real m = M = 0 fields packed in pairs
  P.fkinds.clear();
  P.fcomp.clear();
  std::map<LKey, int> fidx;
  std::vector<LKey> m0l, mpos;
  for (auto& kv : used) {
    const LKey& key = kv.first;
    const LKey base(std::get<0>(key), std::get<1>(key), 0, std::get<3>(key), std::get<4>(key));
    if (std::get<1>(key) == 0 && std::get<4>(key) == 0) {
      m0l.push_back(base);
    } else if (std::find(mpos.begin(), mpos.end(), base) == mpos.end()) {
      mpos.push_back(base);
    }
  }
  for (size_t i = 0; i < m0l.size(); i += 2) {
    FKind k{};
    int la = std::get<0>(m0l[i]);
    cd ca = (la % 2) ? cd(0, -1) : cd(1, 0);
    k.part[0] = FPart{la, 0, ca.real(), ca.imag(), -1, 0};
    source(k.part[0], std::get<3>(m0l[i]), 0);
    k.nparts = 1;
    int kind = (int)P.fkinds.size();
    fidx[m0l[i]] = (int)P.fcomp.size();
    P.fcomp.push_back({kind, 0});
    if (i + 1 < m0l.size()) {
      int lb = std::get<0>(m0l[i + 1]);
      cd cb = ((lb % 2) ? cd(0, -1) : cd(1, 0)) * cd(0, 1);   // i c_lb
      k.part[1] = FPart{lb, 0, cb.real(), cb.imag(), -1, 0};
      source(k.part[1], std::get<3>(m0l[i + 1]), 0);
      k.nparts = 2;
      fidx[m0l[i + 1]] = (int)P.fcomp.size();
      P.fcomp.push_back({kind, 1});
    }
    P.fkinds.push_back(k);
  }
  for (auto& key : mpos) {
    FKind k{};
    k.part[0] = FPart{std::get<0>(key), std::get<1>(key), 1.0, 0.0, -1, 0};
    source(k.part[0], std::get<3>(key), std::get<4>(key));
    k.nparts = 1;
    int kind = (int)P.fkinds.size();
    for (int part = 0; part < 2; ++part) {
      LKey pk(std::get<0>(key), std::get<1>(key), part, std::get<3>(key), std::get<4>(key));
      fidx[pk] = (int)P.fcomp.size();
      P.fcomp.push_back({kind, part});
    }
    P.fkinds.push_back(k);
  }
  P.fsources = false;
  for (auto& k : P.fkinds)
    for (int p = 0; p < k.nparts; ++p) P.fsources = P.fsources || k.part[p].src >= 0;
  // terms sorted by (mu, f2): one Q group per (mu, f2)
  P.terms.clear();
  for (auto& t : kept)
    P.terms.push_back({std::get<0>(t), fidx.at(std::get<1>(t)), fidx.at(std::get<2>(t)),
                       std::get<3>(t), std::get<4>(t)});
  std::sort(P.terms.begin(), P.terms.end(), [](const Term& a, const Term& b) {
    return std::tie(a.mu, a.f2, a.f1, a.g) < std::tie(b.mu, b.f2, b.f1, b.g);
  });
  P.qgroups.clear();
  for (int t = 0; t < (int)P.terms.size(); ++t) {
    if (P.qgroups.empty() || P.qgroups.back().mu != P.terms[t].mu || P.qgroups.back().f2 != P.terms[t].f2)
      P.qgroups.push_back({P.terms[t].mu, P.terms[t].f2, t, t + 1});
    else
      P.qgroups.back().t1 = t + 1;
  }
  // outputs (mu, b1, b2) of the requested pair set
  P.outs.clear();
  P.out_norm.clear();
  const double M3 = (double)P.M * P.M * P.M;
  for (int mu = 0; mu < (int)P.mult.size(); ++mu) {
    int q0 = -1, q1 = -1;
    for (int q = 0; q < (int)P.qgroups.size(); ++q)
      if (P.qgroups[q].mu == mu) {
        if (q0 < 0) q0 = q;
        q1 = q + 1;
      }
    if (q0 < 0) q0 = q1 = 0;   // every term vanishes: B = 0
    bool same = P.mult[mu].l1 == P.mult[mu].l2;
    for (int b1 = 0; b1 < P.nb; ++b1)
      for (int b2 = 0; b2 < P.nb; ++b2) {
        bool want;
        switch (P.pair_mode) {
          case TSB_PAIRS_PAPER: want = same ? (b1 <= b2) : true; break;
          case TSB_PAIRS_UPPER: want = b1 <= b2; break;
          case TSB_PAIRS_DIAGONAL: want = b1 == b2; break;
          default: want = true;
        }
        if (!want || P.nmode[b1] == 0 || P.nmode[b2] == 0) continue;
        P.outs.push_back({mu, b1, b2, q0, q1});
        double nrm = P.mu_pref[mu] / ((double)P.nmode[b1] * (double)P.nmode[b2] * M3);
        // 3PCF: the three fields of eq. 48 carry 1/V each (eqs. 42, 49), of
        // which the estimator's cell volume takes one back
        if (xi) nrm /= P.L * P.L * P.L * P.L * P.L * P.L;
        P.out_norm.push_back(nrm);
      }
  }

  // ---- assignment tile and reduction chunk ---------------------------------------
  // one grid copy's fixed-point words per node sit in LDS at a time
  const int words = assign_words(P);
  if (N % 8 == 0 && N / 8 >= 3 && (int64_t)words * 512 * 8 <= 65536)
    P.T = 8;
  else
    P.T = 4;
  P.NT = N / P.T;
  if ((int64_t)words * P.T * P.T * P.T * 8 > 64 * 1024)
    return fail(TSB_E_UNSUPPORTED, "too many channels for the assignment tile");
  const int esz = P.precision == TSB_FP64 ? 8 : 4;
  const int64_t per_cell = (int64_t)P.nb * (int64_t)P.fcomp.size() + (int64_t)P.gcomp.size() +
                           (int64_t)P.qgroups.size() * P.nb;
  int C = 64;
  while (C > 4 && per_cell * (C + 1) * esz > 65536) C /= 2;
  if (per_cell * (C + 1) * esz > 160 * 1024)
    return fail(TSB_E_UNSUPPORTED, "too many fields for the reduction tile");
  P.red_chunk = C;
  const int64_t nchunks = (int64_t)P.M * P.M * P.M / C;
  P.red_wg = (int)std::min<int64_t>(nchunks, 1024);

  // right factors of the contraction and the fused path
  P.f2idx.assign(P.fcomp.size(), -1);
  P.nf2 = 0;
  for (auto& q : P.qgroups)
    if (P.f2idx[q.f2] < 0) P.f2idx[q.f2] = P.nf2++;
  plan_fused(P);
  P.zcol = !P.assign_tiles && zcol_applies(P);
  if (P.fused && !P.fused_wide) P.red_wg = (int)std::min<int64_t>((int64_t)P.M * P.M, 1024);
  // unfused FP32 plans with at most 32 shells: the sum over a chunk's cells on
  // the matrix cores (32 x 32 tiles, k steps of 8 cells), up to 16 Q groups
  P.red_mfma = 0;
  if (!P.fused && P.precision == TSB_FP32 && P.nb <= 32 && P.red_chunk % 8 == 0 && P.fkinds.size() <= 32 &&
      P.grids.size() <= 32) {   // (unfused_mfma_applies holds the same conditions for the wide kernel)
    const int upw = ((int)P.qgroups.size() + 3) / 4;
    if (upw >= 1 && upw <= 4) P.red_mfma = upw == 1 ? 1 : (upw == 2 ? 2 : 4);
    // fewer, longer chunks: up to 96 KiB of staged rows (one workgroup per CU
    // then; a chunk's fixed costs dominate short ones). Plans whose terms fit
    // the kernel arguments take the 1024-thread kernel with up to 150 KiB.
    if (P.red_mfma) {
      const bool wide = P.qgroups.size() <= 16 && P.terms.size() <= 64;
      if (wide) P.red_mfma = 8;
      const int64_t cap = wide ? 150 * 1024 : 96 * 1024;
      // the 1024-thread kernel stages whole complex rows of every F slot and G grid
      const int64_t cell = wide ? 2 * ((int64_t)P.nb * (int64_t)P.fkinds.size() + (int64_t)P.grids.size()) +
                                      (int64_t)P.qgroups.size() * P.nb
                                : per_cell;
      int Cm = 64;
      while (Cm > 8 && cell * (Cm + 1) * esz > cap) Cm /= 2;
      if (Cm > P.red_chunk) {
        P.red_chunk = Cm;
        P.red_wg = (int)std::min<int64_t>((int64_t)P.M * P.M * P.M / Cm, 1024);
      }
      // two 512-thread workgroups per CU when both sets of staged rows fit its LDS
      P.red_block = reduce_pair_fits(P) ? 512 : 1024;
    }
  }
  P.g_offset = P.fused ? 0 : (int64_t)P.nb * (int64_t)P.fkinds.size() * P.M * P.M * P.M;
  if (P.shot_noise) {
    if (int rc = shot_plan(P)) return rc;
    P.use_graph = false;   // its passes are launched directly
  }
  return TSB_OK;
}

}  // namespace tsb
