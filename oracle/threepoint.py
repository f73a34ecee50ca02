"""FP64 reference of the three-point-function multipoles and of the window
multipoles, plain and slow.

TEST INFRASTRUCTURE ONLY (see the package header).

What it computes (arXiv:1803.02132):

  zeta_{l1 l2 L}(r1, r2)   Sec. 4.3, eq. 47 (definition) and eq. 48 (FFT form)
  Q_{l1 l2 L}(r1, r2)      Sec. 6.1, eq. 58: eq. 47 with dn replaced by the
                           randoms' nbar = alpha sum_ran w delta_D (eq. 32)

Definition on the grid (eq. 47 with the angular averages over r^1 and r^2
taken, like the k-shells of eq. 38, as the mean over the grid separation
vectors r = H n whose length falls in the bin):

  zeta(b1, b2) = (N H_{l1l2L} / I) sum_{m1 m2 M} 3j
                 (1/(N_r(b1) N_r(b2))) sum_{n1 in b1} sum_{n2 in b2}
                 y_l1^m1*(n^1) y_l2^m2*(n^2) v_c sum_x dn(x + H n1) dn(x + H n2) dn_L^M(x),

with dn(x) the deconvolved density field of the grid (its DFT is dn(k) of
estimator.spectra: interlaced, divided by W_mass, Nyquist zeroed) and
v_c = V / N^3. The FFT form of eq. 48 follows by writing the separation average
as a filter in Fourier space:

  F_l^m(x; b) = (1/V) sum_k e^{ik.x} dn(k) K_l^m(k; b),
  K_l^m(k; b) = (1/N_r(b)) sum_{n in b} y_l^m*(n^) e^{ik.Hn},

whose continuum limit is the paper's i^l j_l(kr) y_l^m*(k^) (eq. 49); G_L^M is
the one of eq. 42 over every mode.

Readings:
  T1  r-bins: [r_min + b dr, r_min + (b+1) dr) on |r| = H sqrt(n^2), decided
      once per integer n^2 in FP64 (the k-shell rule of R1 with H for k_f);
      the zero separation n = 0 falls in the bin that holds r = 0, if any, and
      has no direction: its y_l^m is the mean over directions, delta_l0.
      Every bin must lie inside half the box (no separation vector with a
      component N/2), so that r and -r are distinct.
  T2  The separation average is the discrete mean over grid vectors (the
      configuration-space counterpart of eq. 38), not a Bessel filter; the
      two agree in the continuum limit.
  T3  Window multipoles: the channels are built from the randoms alone with
      weight +alpha w y_L^M*(x^) (nbar of eq. 32), galaxies only fix alpha; I is
      the survey normalisation (R8).
  T4  The 3PCF shot noise is the bispectrum's coincident-index terms
      (eqs. 44-46, readings S1-S5 of oracle/shotnoise.py) with the separation
      kernels K in place of the shell filters: the shell averages of y_l^m*
      become Kbar = (1/V) sum_k K_l^m(k; b), which vanishes unless the bin
      holds r = 0 (where only l = 0 survives), the two-point sums become
      (1/V) sum_k K [dn N_L^M* - Sbar C/W^2], and the unit shell fields become
      the kernel fields (1/V) sum_k e^{ik.x} K. For bins without r = 0 only the
      i = j != k term is left, and it lives on b1 = b2: the grid form of eq. 51,
      (N^3/V)(N H/I) sum_m 3j (-1)^{l1+l2} (1/N_r^2) sum_{n in b}
      y_l1^m1*(n^) y_l2^m2*(n^) H_L^M(Hn). The kernels are taken over every
      mode of the grid, Nyquist planes included, so that the kernel fields are
      combs of points at the separation vectors (eq. 51 holds exactly); the
      fields they meet (H, and the two-point spectra dn N_L^M* - Sbar C/W^2 of
      the j = k and i = k terms) are zero on the Nyquist planes like every
      field of the grid (R6). For a bin holding r = 0 the two-point sums are
      (1/(V N_r)) sum_{n in b} y_l^m*(n^) v(Hn), v the inverse transform of the
      two-point spectrum, and Kbar_0^0 = N^3/(V N_r).

Pins (tests/test_oracle_threepoint.py): the FFT form against the direct sum
over grid points and separation vectors above; the Legendre form at L = 0
(eq. 50); the exact value Q_000 = 1 of a uniform density (I = nbar^3 V);
transpose symmetry; the shot noise's i = j != k term against the real-space
form of eq. 51 above, and the vanishing of the other terms and of the
off-diagonal pairs for bins without r = 0.
"""
import numpy as np

from . import angular as ang
from . import estimator as est


def grid_spacing(plan):
    return plan.box_len / plan.n


def r_bin_of_n2(plan):
    """T1: r-bin of every integer n^2 in [0, 3 (N/2)^2]; -1 if none. The plan's
    k_min / dk / edges are read as r_min / dr / r edges (length units)."""
    n2max = 3 * (plan.n // 2) ** 2
    n2 = np.arange(n2max + 1, dtype=np.float64)
    r = grid_spacing(plan) * np.sqrt(n2)
    if plan.edges is None:
        b = np.floor((r - plan.k_min) / plan.dk)
    else:
        e = np.asarray(plan.edges, dtype=np.float64)
        b = np.searchsorted(e, r, side="right") - 1.0
    return np.where((b >= 0) & (b < plan.n_bins), b, -1).astype(np.int64)


def separation_vectors(plan):
    """Integer separation vectors n (signed, (-N/2, N/2]) on the full grid, and
    the r-bin of each; raises if a bin reaches half the box (T1)."""
    nx, ny, nz = est.mode_vectors(plan.n)
    rb = r_bin_of_n2(plan)[nx * nx + ny * ny + nz * nz]
    half = plan.n // 2
    if np.any((rb >= 0) & ((np.abs(nx) == half) | (np.abs(ny) == half) | (np.abs(nz) == half))):
        raise ValueError("an r-bin reaches half the box")
    return nx, ny, nz, rb


def n_r(plan):
    """N_r(b): number of grid separation vectors in each r-bin."""
    rb = separation_vectors(plan)[3]
    return np.array([int(np.sum(rb == b)) for b in range(plan.n_bins)], dtype=np.int64)


def separation_units(nx, ny, nz):
    """n^ of every separation vector and the mask of n = 0 (whose direction is
    arbitrary: sep_ylm_conj gives it delta_l0)."""
    r = np.sqrt(nx * nx + ny * ny + nz * nz).astype(np.float64)
    zero = r == 0
    r[zero] = 1.0
    ux, uy, uz = nx / r, ny / r, nz / r
    uz = np.where(zero, 1.0, uz)
    return ux, uy, uz, zero


def sep_ylm_conj(l, m, ux, uy, uz, zero):
    """y_l^m*(n^) of separation vectors, delta_l0 for n = 0 (T1)."""
    y = np.conj(ang.ylm(l, m, ux, uy, uz))
    return np.where(zero, 1.0 if l == 0 else 0.0, y)


def kernel(plan, l, m, b, sep=None):
    """K_l^m(k; b) on the full grid of modes (T2)."""
    nx, ny, nz, rb = separation_vectors(plan) if sep is None else sep
    ux, uy, uz, zero = separation_units(nx, ny, nz)
    sel = rb == b
    A = np.zeros(nx.shape, dtype=np.complex128)
    A[sel] = sep_ylm_conj(l, m, ux[sel], uy[sel], uz[sel], zero[sel])
    # sum_n A(n) e^{+2 pi i k.n / N} = N^3 ifftn(A)[k]
    return (plan.n ** 3 / np.sum(sel)) * np.fft.ifftn(A)


def reduce_fft(plan, spec, I, pairs=None):
    """eq. 48 on the grid: zeta[mu][b1][b2] (real part) and its imaginary part."""
    n = plan.n
    nb = plan.n_bins
    sep = separation_vectors(plan)
    if pairs is None:
        pairs = [(b1, b2) for b1 in range(nb) for b2 in range(nb)]
    pairs = list(pairs)
    dv = plan.volume / n ** 3
    out_re = np.full((len(plan.multipoles), nb, nb), np.nan)
    out_im = np.full((len(plan.multipoles), nb, nb), np.nan)
    fcache, gcache = {}, {}

    def F(l, m, b):
        if (l, m, b) not in fcache:
            fcache[(l, m, b)] = (n ** 3 / plan.volume) * np.fft.ifftn(spec[(0, 0)] * kernel(plan, l, m, b, sep))
        return fcache[(l, m, b)]

    def G(L, M):
        if (L, M) not in gcache:
            gcache[(L, M)] = est.g_field(plan, spec, L, M)
        return gcache[(L, M)]

    for mu, (l1, l2, L) in enumerate(plan.multipoles):
        terms = ang.reduction_terms(l1, l2, L, los="local")
        pref = ang.n_factor(l1, l2, L) * ang.h_factor(l1, l2, L) / I
        for (b1, b2) in pairs:
            acc = 0j
            for (m1, m2, M, w3j) in terms:
                acc += w3j * dv * np.sum(F(l1, m1, b1) * F(l2, m2, b2) * G(L, M))
            out_re[mu, b1, b2] = (pref * acc).real
            out_im[mu, b1, b2] = (pref * acc).imag
    return out_re, out_im


def direct_sum(plan, spec, I, pairs=None):
    """eq. 47 on the grid, literally: for every pair of separation vectors of
    the two bins, v_c sum_x dn(x + H n1) dn(x + H n2) dn_L^M(x) (shifts of the
    periodic grid), weighted by y_l1^m1*(n^1) y_l2^m2*(n^2) and 3j."""
    n = plan.n
    nb = plan.n_bins
    nx, ny, nz, rb = separation_vectors(plan)
    ux, uy, uz, zero = separation_units(nx, ny, nz)
    dens = {k: (n ** 3 / plan.volume) * np.fft.ifftn(v) for k, v in spec.items()}   # dn(x)
    d0 = dens[(0, 0)]
    if pairs is None:
        pairs = [(b1, b2) for b1 in range(nb) for b2 in range(nb)]
    dv = plan.volume / n ** 3
    vecs = {}
    for b in range(nb):
        sel = np.nonzero(rb == b)
        vecs[b] = (nx[sel], ny[sel], nz[sel], ux[sel], uy[sel], uz[sel], zero[sel])
    out = np.full((len(plan.multipoles), nb, nb), np.nan)
    for mu, (l1, l2, L) in enumerate(plan.multipoles):
        terms = ang.reduction_terms(l1, l2, L, los="local")
        pref = ang.n_factor(l1, l2, L) * ang.h_factor(l1, l2, L) / I
        for (b1, b2) in pairs:
            v1, v2 = vecs[b1], vecs[b2]
            shift1 = [np.roll(d0, (-a, -b, -c), axis=(0, 1, 2)) for a, b, c in zip(v1[0], v1[1], v1[2])]
            shift2 = [np.roll(d0, (-a, -b, -c), axis=(0, 1, 2)) for a, b, c in zip(v2[0], v2[1], v2[2])]
            acc = 0j
            for (m1, m2, M, w3j) in terms:
                if plan.los == "global":
                    d = np.asarray(plan.los_dir, np.float64)
                    d = d / np.linalg.norm(d)
                    g = complex(np.conj(ang.ylm(L, M, d[0], d[1], d[2]))) * d0
                else:
                    g = dens[(L, M)]
                y1 = sep_ylm_conj(l1, m1, v1[3], v1[4], v1[5], v1[6])
                y2 = sep_ylm_conj(l2, m2, v2[3], v2[4], v2[5], v2[6])
                a1 = sum(y * s for y, s in zip(y1, shift1)) / len(y1)   # separation average, dn(x + H n1)
                a2 = sum(y * s for y, s in zip(y2, shift2)) / len(y2)
                acc += w3j * dv * np.sum(a1 * a2 * g)
            out[mu, b1, b2] = (pref * acc).real
    return out


def window_spectra(plan, data, randoms):
    """T3: the channels of nbar = alpha sum_ran w y_L^M*(x^) delta_D, gridded and
    transformed like dn (O4-O6); returns (spectra, I, alpha)."""
    if plan.box_mode:
        raise ValueError("window multipoles need a random catalogue (survey mode)")
    pos = np.asarray(data["pos"], np.float64)
    w_c = data.get("w")
    w = est.fkp_weights(np.ones(len(pos)) if w_c is None else w_c, data.get("nbar"), plan.P0)
    rpos = np.asarray(randoms["pos"], np.float64)
    rw_c = randoms.get("w")
    rw = est.fkp_weights(np.ones(len(rpos)) if rw_c is None else rw_c, randoms.get("nbar"), plan.P0)
    alpha = est.alpha_ratio(w, rw)
    shifts = [0.0, 0.5] if plan.interlace else [0.0]
    grids = {}
    for (L, M) in est.channels(plan):
        grids[(L, M)] = [alpha * est.assign(rpos, est.channel_weights(rpos, rw, L, M, plan), plan, shift=s)
                         for s in shifts]
    spec = est.spectra(plan, grids)
    R = est.assign(rpos, rw, plan, shift=0.0).real
    vc = plan.volume / plan.n ** 3
    I = float(np.sum((alpha * R) ** 3) / vc ** 2)   # R8, eq. 37
    return spec, I, alpha


def measure(plan, data, randoms=None, pairs=None, window=False):
    """zeta (eq. 48) end to end, or Q (eq. 58) with window=True."""
    if window:
        spec, I, alpha = window_spectra(plan, data, randoms)
    else:
        grids, info = est.assign_channels(plan, data, randoms)
        spec = est.spectra(plan, grids)
        I, alpha = info["I"], info["alpha"]
    zr, zi = reduce_fft(plan, spec, I, pairs=pairs)
    return {"zeta": zr, "zeta_imag": zi, "I": I, "alpha": alpha, "n_r": n_r(plan), "spectra": spec}


def two_point_spectrum(plan, spec, nk, sb, cw2, L, M):
    """dn(k) N_L^M*(k) - Sbar_L^M C(k)/W^2(k), zero on the Nyquist planes (T4, R6)."""
    n = plan.n
    nx, ny, nz = est.mode_vectors(n)
    v = spec[(0, 0)] * np.conj(nk[(L, M)]) - sb[(L, M)] * cw2
    v[(np.abs(nx) == n // 2) | (np.abs(ny) == n // 2) | (np.abs(nz) == n // 2)] = 0.0
    return v


def two_point_sum(plan, spec, nk, sb, cw2, Kb, L, M):
    """(1/V) sum_k K(k; b) [dn N_L^M* - Sbar C/W^2](k) for the kernel Kb (T4)."""
    return complex(np.sum(Kb * two_point_spectrum(plan, spec, nk, sb, cw2, L, M)) / plan.volume)


def shot_noise(plan, spec, nk, sb, cw2, I, pairs=None):
    """T4: the four coincident-index terms with separation kernels. Arguments as
    shotnoise.shot_noise (spec: dn_L^M(k), nk: N_L^M(k), sb: Sbar_L^M, cw2: C/W^2).
    Returns dict of (n_mult, n_bins, n_bins) arrays 'iii', 'jk', 'ik', 'ij', 'S'."""
    n = plan.n
    nb = plan.n_bins
    sep = separation_vectors(plan)
    if pairs is None:
        pairs = [(b1, b2) for b1 in range(nb) for b2 in range(nb)]
    pairs = list(pairs)
    nmult = len(plan.multipoles)
    out = {k: np.full((nmult, nb, nb), np.nan) for k in ("iii", "jk", "ik", "ij", "S")}
    dv = plan.volume / n ** 3
    nx, ny, nz = est.mode_vectors(n)
    nyq = (np.abs(nx) == n // 2) | (np.abs(ny) == n // 2) | (np.abs(nz) == n // 2)
    kc, hc = {}, {}

    def K(l, m, b):
        if (l, m, b) not in kc:
            kc[(l, m, b)] = kernel(plan, l, m, b, sep)
        return kc[(l, m, b)]

    def Kbar(l, m, b):
        return complex(np.sum(K(l, m, b)) / plan.volume)

    def A(l, m, L, M, b):
        return two_point_sum(plan, spec, nk, sb, cw2, K(l, m, b), L, M)

    def f(l, m, b):
        return (n ** 3 / plan.volume) * np.fft.ifftn(K(l, m, b))

    def H(L, M):
        if (L, M) not in hc:
            src = spec[(L, M)] if (L, M) in spec else None
            if src is None:   # global LOS (R10)
                d = np.asarray(plan.los_dir, np.float64)
                d = d / np.linalg.norm(d)
                src = complex(np.conj(ang.ylm(L, M, d[0], d[1], d[2]))) * spec[(0, 0)]
            h = src * np.conj(nk[(0, 0)]) - sb[(L, M)] * cw2
            h[nyq] = 0.0
            hc[(L, M)] = (n ** 3 / plan.volume) * np.fft.ifftn(h)
        return hc[(L, M)]

    for mu, (l1, l2, L) in enumerate(plan.multipoles):
        terms = ang.reduction_terms(l1, l2, L, los="local")
        pref = ang.n_factor(l1, l2, L) * ang.h_factor(l1, l2, L) / I
        for (b1, b2) in pairs:
            t = {"iii": 0j, "jk": 0j, "ik": 0j, "ij": 0j}
            for (m1, m2, M, w3j) in terms:
                t["iii"] += w3j * Kbar(l1, m1, b1) * Kbar(l2, m2, b2) * sb[(L, M)]
                t["jk"] += w3j * A(l1, m1, L, M, b1) * Kbar(l2, m2, b2)
                t["ik"] += w3j * Kbar(l1, m1, b1) * A(l2, m2, L, M, b2)
                t["ij"] += w3j * dv * np.sum(f(l1, m1, b1) * f(l2, m2, b2) * H(L, M))
            for k in t:
                out[k][mu, b1, b2] = (pref * t[k]).real
            out["S"][mu, b1, b2] = sum(out[k][mu, b1, b2] for k in ("iii", "jk", "ik", "ij"))
    return out


def shot_noise_eq51(plan, spec, nk, sb, cw2, I):
    """The grid form of eq. 51 for bins without r = 0: diagonal pairs only,
    (N^3/V)(N H/I) sum_m 3j (-1)^{l1+l2} (1/N_r^2) sum_{n in b} y* y* H_L^M(Hn),
    H evaluated at the grid point of each separation vector (T4)."""
    n = plan.n
    nx, ny, nz, rb = separation_vectors(plan)
    ux, uy, uz, zero = separation_units(nx, ny, nz)
    mnx, mny, mnz = est.mode_vectors(n)
    nyq = (np.abs(mnx) == n // 2) | (np.abs(mny) == n // 2) | (np.abs(mnz) == n // 2)
    out = np.full((len(plan.multipoles), plan.n_bins, plan.n_bins), np.nan)
    for mu, (l1, l2, L) in enumerate(plan.multipoles):
        pref = ang.n_factor(l1, l2, L) * ang.h_factor(l1, l2, L) / I
        for b in range(plan.n_bins):
            sel = np.nonzero(rb == b)
            if len(sel[0]) == 0:
                continue
            tot = 0j
            for (m1, m2, M, w3j) in ang.reduction_terms(l1, l2, L, los="local"):
                if (L, M) in spec:
                    src = spec[(L, M)]
                else:   # global LOS (R10)
                    d = np.asarray(plan.los_dir, np.float64)
                    d = d / np.linalg.norm(d)
                    src = complex(np.conj(ang.ylm(L, M, d[0], d[1], d[2]))) * spec[(0, 0)]
                h = src * np.conj(nk[(0, 0)]) - sb[(L, M)] * cw2
                h[nyq] = 0.0
                Hx = (n ** 3 / plan.volume) * np.fft.ifftn(h)
                y1 = sep_ylm_conj(l1, m1, ux[sel], uy[sel], uz[sel], zero[sel])
                y2 = sep_ylm_conj(l2, m2, ux[sel], uy[sel], uz[sel], zero[sel])
                hv = Hx[nx[sel] % n, ny[sel] % n, nz[sel] % n]
                tot += w3j * np.sum(y1 * y2 * hv)
            val = (n ** 3 / plan.volume) * pref * (-1) ** (l1 + l2) * tot / len(sel[0]) ** 2
            out[mu, b, b] = val.real
    return out


def measure_shot_noise(plan, data, randoms=None, pairs=None):
    """zeta (eq. 48) and its shot noise (T4) end to end; zeta - S is the
    shot-noise-subtracted multipole."""
    from . import shotnoise as sn
    res = measure(plan, data, randoms, pairs=pairs)
    nk = sn.n_spectra(plan, data, randoms)
    sb = sn.sbar(plan, data, randoms)
    out = shot_noise(plan, res["spectra"], nk, sb, sn.shot_window(plan), res["I"], pairs=pairs)
    out["zeta"] = res["zeta"]
    out["I"] = res["I"]
    out["alpha"] = res["alpha"]
    return out
