"""FP64 reference of the shot noise of the bispectrum-multipole estimator.

TEST INFRASTRUCTURE ONLY (see the package header).

What it computes (arXiv:1803.02132, Sec. 4.2, eqs. 43-46). Writing the
estimator in the particle description (eq. 43), a triple sum over particles
i, j, k (galaxies, and randoms weighted by -alpha), the shot noise is the part
of that sum where indices coincide (eq. 44):

  S = S|_{i=j=k} + S|_{i=j!=k} + S|_{i=k!=j} + S|_{j=k!=i},

each term built from (eq. 46)

  Sbar_L^M = (sum_gal - alpha^3 sum_ran) w^3 y_L^M*(x^),
  N_L^M(k) = (sum_gal + alpha^2 sum_ran) w^2 y_L^M(x^) e^{-ik.x}.

On the grid every shell average is the discrete mode sum of eq. 38, so the
four terms of eq. 45 read, with C(k) the alias sum of W_mass^2 (below):

  S|_{i=j=k}    = (N H / I) sum_m 3j ybar_l1^m1*(b1) ybar_l2^m2*(b2) Sbar_L^M
  S|_{j=k!=i}   = (N H / I) sum_m 3j A_{l1 m1}^{L M}(b1) ybar_l2^m2*(b2)
  S|_{i=k!=j}   = (N H / I) sum_m 3j ybar_l1^m1*(b1) A_{l2 m2}^{L M}(b2)
  S|_{i=j!=k}   = (N H / I) sum_m 3j (V/N^3) sum_x f_l1^m1(x;b1) f_l2^m2(x;b2) H_L^M(x)

  ybar_l^m*(b)      = (1/N_mode) sum_{k in b} y_l^m*(k^)
  A_{l m}^{L M}(b)  = (1/N_mode) sum_{k in b} y_l^m*(k^) [dn(k) N_L^M*(k) - Sbar_L^M C(k)/W^2(k)]
  f_l^m(x; b)       = (1/N_mode) sum_{k in b} y_l^m*(k^) e^{ik.x}
  H_L^M(x)          = (1/V) sum_k e^{ik.x} [dn_L^M(k) N_0^0*(k) - Sbar_L^M C(k)/W^2(k)]

Readings (the paper's printed forms are the continuum limits of these):
  S1  The paper's Kronecker deltas (l1 = 0 in S|_{i=k!=j} and so on) come from
      continuous shell averages of y_l^m; the lattice average ybar is kept,
      which equals delta_{l0} exactly for l <= 3 and differs for l >= 4 (the
      cubic lattice has an invariant combination at l = 4).
  S2  The paper's i^{l1+l2} j_l1(k1 x) j_l2(k2 x) y_l1^m1*(x^) y_l2^m2*(x^) is the
      continuum value of f_l1^m1(x; k1) f_l2^m2(x; k2); the discrete f is used
      (the same shell sums as the F fields of eq. 42), and the free index M of
      the two-point terms is summed with the 3j weights.
  S3  C(k) (the paper cites Jing 2005, eq. 20, not reproduced in it) is taken
      as the exact alias sum the subtraction stands for: the expected
      self-pair term of dn(k) N*(k) for particles placed uniformly in a cell,
        C(k) = sum_n W^2(k + 2 k_N n)                    (no interlacing),
        C(k) = sum_{n: nx+ny+nz even} W^2(k + 2 k_N n)    (interlaced grids),
      with W the order-p kernel per axis; per axis with x = pi n_a / N,
        A_p = sum_n sinc^{2p}(x + pi n):  1, 1 - (2/3) s^2, 1 - s^2 + (2/15) s^4,
        B_p = sum_n (-1)^n sinc^{2p}(x + pi n): cos x, (cos^3 x + 5 cos x)/6,
              (cos^5 x + 58 cos^3 x + 61 cos x)/120,
      s = sin x, so that C = prod A_p, or (prod A_p + prod B_p)/2 interlaced.
  S4  S|_{i=j=k} carries no such correction, as in the paper (it says the
      scale dependence of this term is left for future work).
  S5  N_L^M is a pure particle sum: in a periodic box it has no mean term and
      no randoms, and its DC mode is kept; it is gridded, interlaced,
      deconvolved and Nyquist-zeroed like dn. H_L^M is zero on the Nyquist
      planes too (R6 for every field: dn and N vanish there, and so does the
      self-pair part of their product that the subtraction stands for).

Pins (tests/test_oracle_shotnoise.py): the terms against a direct triple sum
over particle indices split by coincidence class, with exact particle Fourier
sums (W = C = 1); C against truncated alias sums; S|_{i=j=k} and the box-mode
DC identity; the paper's Kronecker-delta forms for l <= 3.
"""
import numpy as np

from . import angular as ang
from . import estimator as est


# ----------------------------------------------------------------------------
# alias sums of the assignment window (reading S3)


def alias_sums(p, x):
    """Per-axis A_p(x) = sum_n sinc^{2p}(x + pi n) and B_p(x) = sum_n (-1)^n sinc^{2p}(x + pi n)
    in closed form (derivatives of cot and csc at x), sinc(t) = sin t / t."""
    x = np.asarray(x, dtype=np.float64)
    s2 = np.sin(x) ** 2
    c = np.cos(x)
    if p == 1:
        return np.ones_like(x), c
    if p == 2:
        return 1.0 - 2.0 / 3.0 * s2, (c ** 3 + 5.0 * c) / 6.0
    if p == 3:
        return 1.0 - s2 + 2.0 / 15.0 * s2 * s2, (c ** 5 + 58.0 * c ** 3 + 61.0 * c) / 120.0
    raise ValueError("assign_p must be 1, 2 or 3")


def shot_window(plan):
    """C(k) / W_mass^2(k) on the full grid (reading S3)."""
    nx, ny, nz = est.mode_vectors(plan.n)
    per = [alias_sums(plan.assign_p, np.pi * v / plan.n) for v in (nx, ny, nz)]
    C = per[0][0] * per[1][0] * per[2][0]
    if plan.interlace:
        C = 0.5 * (C + per[0][1] * per[1][1] * per[2][1])
    return C / est.mass_window(plan) ** 2


# ----------------------------------------------------------------------------
# eq. 46: the scalars Sbar and the w^2-weighted fields N


def _weights(plan, data, randoms):
    pos = np.asarray(data["pos"], np.float64)
    w_c = data.get("w")
    w = est.fkp_weights(np.ones(len(pos)) if w_c is None else w_c, data.get("nbar"), plan.P0)
    if plan.box_mode:
        return pos, w, None, None, 0.0
    rpos = np.asarray(randoms["pos"], np.float64)
    rw_c = randoms.get("w")
    rw = est.fkp_weights(np.ones(len(rpos)) if rw_c is None else rw_c, randoms.get("nbar"), plan.P0)
    return pos, w, rpos, rw, est.alpha_ratio(w, rw)


def _ylm_conj(plan, pos, L, M):
    """y_L^M*(x^) per particle (local LOS), or y_L^M*(d) (global LOS, R10)."""
    if plan.los == "global":
        d = np.asarray(plan.los_dir, np.float64)
        d = d / np.linalg.norm(d)
        return np.full(len(pos), complex(np.conj(ang.ylm(L, M, d[0], d[1], d[2]))))
    u = est.los_unit_vectors(pos, plan.observer)
    return np.conj(ang.ylm(L, M, u[:, 0], u[:, 1], u[:, 2]))


def sbar(plan, data, randoms=None):
    """Sbar_L^M = (sum_gal - alpha^3 sum_ran) w^3 y_L^M*(x^) for every (L, M) of
    the plan's channels (eq. 46)."""
    pos, w, rpos, rw, alpha = _weights(plan, data, randoms)
    out = {}
    for (L, M) in sorted({(L, M) for L in {mp[2] for mp in plan.multipoles} | {0} for M in range(-L, L + 1)}):
        v = np.sum(w ** 3 * _ylm_conj(plan, pos, L, M))
        if rpos is not None:
            v -= alpha ** 3 * np.sum(rw ** 3 * _ylm_conj(plan, rpos, L, M))
        out[(L, M)] = complex(v)
    return out


def n_spectra(plan, data, randoms=None):
    """N_L^M(k) (eq. 46) for every (L, M) of the plan's channels, gridded like
    dn (O4-O6, interlaced and deconvolved, Nyquist zeroed) without a mean term
    and with its DC mode (reading S5). The particle weights are
    w^2 y_L^M(x^) (galaxies) and alpha^2 w^2 y_L^M(x^) (randoms)."""
    pos, w, rpos, rw, alpha = _weights(plan, data, randoms)
    n = plan.n
    nx, ny, nz = est.mode_vectors(n)
    W = est.mass_window(plan)
    nyq = (np.abs(nx) == n // 2) | (np.abs(ny) == n // 2) | (np.abs(nz) == n // 2)
    shifts = [0.0, 0.5] if plan.interlace else [0.0]
    Ls = sorted({mp[2] for mp in plan.multipoles} | {0}) if plan.los == "local" else [0]
    out = {}
    for L in Ls:
        for M in range(-L, L + 1):
            per = []
            for s in shifts:
                D = est.assign(pos, w ** 2 * np.conj(_ylm_conj(plan, pos, L, M)), plan, shift=s)
                if rpos is not None:
                    D = D + alpha ** 2 * est.assign(rpos, rw ** 2 * np.conj(_ylm_conj(plan, rpos, L, M)), plan,
                                                   shift=s)
                per.append(np.fft.fftn(D))
            S = per[0]
            if plan.interlace:
                S = 0.5 * (S + np.exp(1j * np.pi * (nx + ny + nz) / n) * per[1])
            S = S / W
            S[nyq] = 0.0
            out[(L, M)] = S
    if plan.los == "global":
        # R10: N_L^M = y_L^M(d) N_0^0 (the weight y_L^M(d) is common to all particles)
        d = np.asarray(plan.los_dir, np.float64)
        d = d / np.linalg.norm(d)
        for L in sorted({mp[2] for mp in plan.multipoles}):
            for M in range(-L, L + 1):
                out[(L, M)] = complex(ang.ylm(L, M, d[0], d[1], d[2])) * out[(0, 0)]
    return out


# ----------------------------------------------------------------------------
# eq. 45: the four terms


def shell_average_y(plan, l, m, b, bg=None, units=None):
    """ybar_l^m*(b) = (1/N_mode) sum_{k in b} y_l^m*(k^) (reading S1)."""
    bg = est.bin_grid(plan) if bg is None else bg
    ux, uy, uz = est.mode_unit_vectors(plan) if units is None else units
    sel = bg == b
    if not np.any(sel):
        return 0j
    return complex(np.mean(np.conj(ang.ylm(l, m, ux[sel], uy[sel], uz[sel]))))


def unit_field(plan, l, m, b, bg=None, units=None, nm=None):
    """f_l^m(x; b) = (1/N_mode) sum_{k in b} y_l^m*(k^) e^{ik.x} (reading S2):
    the F field of eq. 42 with dn/W replaced by 1."""
    n = plan.n
    bg = est.bin_grid(plan) if bg is None else bg
    ux, uy, uz = est.mode_unit_vectors(plan) if units is None else units
    nm = est.nmode(plan) if nm is None else nm
    sel = bg == b
    A = np.zeros((n, n, n), dtype=np.complex128)
    A[sel] = np.conj(ang.ylm(l, m, ux[sel], uy[sel], uz[sel]))
    return (n ** 3 / nm[b]) * np.fft.ifftn(A)


def shot_noise(plan, dn, nk, sb, cw2, I, pairs=None):
    """The four terms of eq. 45 on the grid.

    dn:  dict (L, M) -> dn_L^M(k) on the full grid (as est.spectra returns);
    nk:  dict (L, M) -> N_L^M(k) (as n_spectra returns);
    sb:  dict (L, M) -> Sbar_L^M (as sbar returns);
    cw2: C(k)/W^2(k) on the full grid (shot_window; ones for exact particle sums);
    I:   the normalisation.
    Returns a dict of (n_mult, n_bins, n_bins) real arrays: 'iii' (i = j = k),
    'jk' (j = k != i), 'ik' (i = k != j), 'ij' (i = j != k) and 'S', their sum;
    pairs outside `pairs` stay NaN."""
    n = plan.n
    nb = plan.n_bins
    bg = est.bin_grid(plan)
    units = est.mode_unit_vectors(plan)
    nm = est.nmode(plan)
    if pairs is None:
        pairs = [(b1, b2) for b1 in range(nb) for b2 in range(nb)]
    pairs = list(pairs)
    nmult = len(plan.multipoles)
    out = {k: np.full((nmult, nb, nb), np.nan) for k in ("iii", "jk", "ik", "ij", "S")}
    dv = plan.volume / n ** 3
    ybar = {}

    def yb(l, m, b):
        if (l, m, b) not in ybar:
            ybar[(l, m, b)] = shell_average_y(plan, l, m, b, bg, units)
        return ybar[(l, m, b)]

    acache = {}

    def A(l, m, L, M, b):
        """(1/N_mode) sum_{k in b} y_l^m*(k^) [dn(k) N_L^M*(k) - Sbar_L^M C/W^2]."""
        key = (l, m, L, M, b)
        if key not in acache:
            sel = bg == b
            y = np.conj(ang.ylm(l, m, units[0][sel], units[1][sel], units[2][sel]))
            v = dn[(0, 0)][sel] * np.conj(nk[(L, M)][sel]) - sb[(L, M)] * cw2[sel]
            acache[key] = complex(np.sum(y * v) / nm[b])
        return acache[key]

    hcache = {}
    nx, ny, nz = est.mode_vectors(n)
    nyq = (np.abs(nx) == n // 2) | (np.abs(ny) == n // 2) | (np.abs(nz) == n // 2)

    def H(L, M):
        """H_L^M(x) = (N^3/V) ifftn(dn_L^M N_0^0* - Sbar_L^M C/W^2), zero on the
        Nyquist planes like every field (R6; dn and N vanish there, and so does
        the self-pair part of their product)."""
        if (L, M) not in hcache:
            src = dn[(L, M)] if (L, M) in dn else None
            if src is None:   # global LOS: dn_L^M = y_L^M*(d) dn (R10)
                d = np.asarray(plan.los_dir, np.float64)
                d = d / np.linalg.norm(d)
                src = complex(np.conj(ang.ylm(L, M, d[0], d[1], d[2]))) * dn[(0, 0)]
            spec = src * np.conj(nk[(0, 0)]) - sb[(L, M)] * cw2
            spec[nyq] = 0.0
            hcache[(L, M)] = (n ** 3 / plan.volume) * np.fft.ifftn(spec)
        return hcache[(L, M)]

    for mu, (l1, l2, L) in enumerate(plan.multipoles):
        terms = ang.reduction_terms(l1, l2, L, los="local")
        pref = ang.n_factor(l1, l2, L) * ang.h_factor(l1, l2, L) / I
        fcache = {}

        def f(l, m, b):
            if (l, m, b) not in fcache:
                fcache[(l, m, b)] = unit_field(plan, l, m, b, bg, units, nm)
            return fcache[(l, m, b)]

        for (b1, b2) in pairs:
            t = {"iii": 0j, "jk": 0j, "ik": 0j, "ij": 0j}
            for (m1, m2, M, w3j) in terms:
                t["iii"] += w3j * yb(l1, m1, b1) * yb(l2, m2, b2) * sb[(L, M)]
                t["jk"] += w3j * A(l1, m1, L, M, b1) * yb(l2, m2, b2)
                t["ik"] += w3j * yb(l1, m1, b1) * A(l2, m2, L, M, b2)
                t["ij"] += w3j * dv * np.sum(f(l1, m1, b1) * f(l2, m2, b2) * H(L, M))
            for k in t:
                out[k][mu, b1, b2] = (pref * t[k]).real
            out["S"][mu, b1, b2] = sum(out[k][mu, b1, b2] for k in ("iii", "jk", "ik", "ij"))
    return out


def measure_shot_noise(plan, data, randoms=None, pairs=None):
    """eqs. 44-46 end to end on the grid: the terms and their sum S, and the
    raw estimator B of eq. 41 (est.measure) for the same pairs; B - S is the
    shot-noise-subtracted multipole."""
    res = est.measure(plan, data, randoms, pairs=pairs)
    nk = n_spectra(plan, data, randoms)
    sb = sbar(plan, data, randoms)
    sn = shot_noise(plan, res["spectra"], nk, sb, shot_window(plan), res["I"], pairs=pairs)
    sn["B"] = res["B"]
    sn["I"] = res["I"]
    sn["alpha"] = res["alpha"]
    return sn
