"""Pins of the oracle's shot noise (no GPU).

* The four terms of eq. 45 against a direct triple sum over particle indices
  (eq. 43) split by which indices coincide (eq. 44), with exact particle
  Fourier sums (no assignment, so W = C = 1): every term to rounding, and the
  raw estimator minus S equals the sum over distinct triples.
* The alias sums C of W^2 against truncated sums over aliases.
* The paper's printed forms (eq. 45 with Kronecker deltas) for l <= 3.
"""
import math

import numpy as np
import pytest

from oracle import angular as ang
from oracle import estimator as est
from oracle import shotnoise as sn


def _exact_spectra(plan, parts, weight):
    """dict (L, M) -> sum_i weight(i, L, M) e^{-ik.x_i} on the full grid."""
    nx, ny, nz = est.mode_vectors(plan.n)
    k = plan.k_f * np.stack([nx, ny, nz], axis=-1)
    out = {}
    for (L, M) in est.channels(plan):
        acc = np.zeros(nx.shape, dtype=np.complex128)
        for i, x in enumerate(parts["pos"]):
            acc += weight(i, L, M) * np.exp(-1j * (k @ x))
        out[(L, M)] = acc
    return out


def _particles(plan, seed, n_gal, n_ran):
    rng = np.random.default_rng(seed)
    pos = plan.box_len * (0.15 + 0.7 * rng.random((n_gal + n_ran, 3)))
    w = 0.5 + rng.random(n_gal + n_ran)
    ran = np.arange(n_gal + n_ran) >= n_gal
    alpha = w[~ran].sum() / w[ran].sum()
    sign = np.where(ran, -alpha, 1.0)
    u = est.los_unit_vectors(pos, plan.observer)
    return {"pos": pos, "w": w, "ran": ran, "alpha": alpha, "sign": sign, "u": u}


def _c(p, i, L, M):
    """Channel weight c_i^{LM} = (1 or -alpha) w_i y_L^M*(x^_i) (eq. 34)."""
    return p["sign"][i] * p["w"][i] * complex(np.conj(ang.ylm(L, M, *p["u"][i])))


def test_terms_equal_the_coincident_index_parts_of_the_triple_sum():
    # 16^3 periodic grid, shells inside |n| < 4 (so that no triangle wraps and
    # every FFT form is exact), 7 galaxies and 5 randoms with weights
    plan = est.Plan(n=16, box_len=100.0, multipoles=[(0, 0, 0), (2, 0, 2), (1, 1, 0), (1, 1, 2), (4, 0, 4)],
                    n_bins=2, dk=1.4 * 2 * math.pi / 100.0, k_min=0.9 * 2 * math.pi / 100.0, los="local",
                    observer=(50.0, 50.0, -120.0), box_mode=False)
    bg = est.bin_grid(plan)
    nx, ny, nz = est.mode_vectors(plan.n)
    assert np.max(np.abs(np.stack([nx, ny, nz])[:, bg >= 0])) < plan.n // 4
    p = _particles(plan, 5, 7, 5)
    npart = len(p["pos"])
    dn = _exact_spectra(plan, p, lambda i, L, M: _c(p, i, L, M))
    # N_L^M = sum (1 for galaxies, alpha^2 for randoms) w^2 y_L^M(x^) e^{-ik.x}
    nk = _exact_spectra(plan, p, lambda i, L, M: p["sign"][i] ** 2 * p["w"][i] ** 2
                        * complex(ang.ylm(L, M, *p["u"][i])))
    sb = {(L, M): sum(p["sign"][i] ** 3 * p["w"][i] ** 3 * complex(np.conj(ang.ylm(L, M, *p["u"][i])))
                      for i in range(npart)) for (L, M) in est.channels(plan)}
    I = 1.0
    got = sn.shot_noise(plan, dn, nk, sb, np.ones(bg.shape), I)
    raw, _ = est.reduce_fft(plan, dn, I)

    # the direct triple sum over (i, j, k), split by coincidence class
    ii, jj, kk = np.meshgrid(np.arange(npart), np.arange(npart), np.arange(npart), indexing="ij")
    classes = {"iii": (ii == jj) & (jj == kk), "ij": (ii == jj) & (ii != kk), "jk": (jj == kk) & (ii != jj),
               "ik": (ii == kk) & (ii != jj), "distinct": (ii != jj) & (jj != kk) & (ii != kk)}
    ux, uy, uz = est.mode_unit_vectors(plan)
    shells = {}
    for b in range(plan.n_bins):
        sel = np.nonzero(bg == b)
        kv = plan.k_f * np.stack([nx[sel], ny[sel], nz[sel]], axis=1)
        E = np.exp(-1j * (p["pos"] @ kv.T))                       # [particle, mode]
        shells[b] = (E, ux[sel], uy[sel], uz[sel])
    for mu, (l1, l2, L) in enumerate(plan.multipoles):
        pref = ang.n_factor(l1, l2, L) * ang.h_factor(l1, l2, L) / I
        for b1 in range(plan.n_bins):
            for b2 in range(plan.n_bins):
                E1, x1, y1, z1 = shells[b1]
                E2, x2, y2, z2 = shells[b2]
                E3 = np.conj(E1[:, :, None] * E2[:, None, :])      # e^{-i k3.x}, k3 = -k1-k2
                tot = {c: 0j for c in classes}
                for (m1, m2, M, w3j) in ang.reduction_terms(l1, l2, L):
                    u0 = np.array([_c(p, i, 0, 0) for i in range(npart)])
                    v = np.array([_c(p, i, L, M) for i in range(npart)])
                    Y1 = np.conj(ang.ylm(l1, m1, x1, y1, z1))
                    Y2 = np.conj(ang.ylm(l2, m2, x2, y2, z2))
                    for c, mask in classes.items():
                        wgt = mask * u0[:, None, None] * u0[None, :, None] * v[None, None, :]
                        T = np.einsum("ijk,ia,jc,kac->ac", wgt, E1, E2, E3, optimize=True)
                        tot[c] += w3j * np.sum(Y1[:, None] * Y2[None, :] * T) / (len(x1) * len(x2))
                scale = abs(raw[mu, b1, b2]) + sum(abs(pref * t) for t in tot.values())
                for c in ("iii", "ij", "jk", "ik"):
                    assert abs(got[c][mu, b1, b2] - (pref * tot[c]).real) <= 1e-11 * scale, (mu, b1, b2, c)
                # raw estimator = every triple; minus S leaves the distinct ones
                assert abs(raw[mu, b1, b2] - got["S"][mu, b1, b2] - (pref * tot["distinct"]).real) <= 1e-11 * scale


@pytest.mark.parametrize("p", [1, 2, 3])
def test_alias_sums_against_truncated_series(p):
    x = np.array([0.0, 0.1, 0.4, 0.9, 1.3, 1.5])
    A, B = sn.alias_sums(p, x)
    K = 20000
    n = np.arange(-K, K + 1)[:, None]
    t = x[None, :] + np.pi * n
    with np.errstate(invalid="ignore", divide="ignore"):
        sinc = np.where(t == 0.0, 1.0, np.sin(t) / t)
    a = np.sum(sinc ** (2 * p), axis=0)
    b = np.sum((-1.0) ** n * sinc ** (2 * p), axis=0)
    if p == 1:
        # the tails beyond |n| = K: sum_{|n|>K} sin^2 x/(pi n)^2 ~ 2 sin^2 x/(pi^2 K) (A);
        # they cancel to O(K^-2) in the alternating sum (B)
        a += 2.0 * np.sin(x) ** 2 / (np.pi ** 2 * K)
        assert np.allclose(A, a, rtol=0, atol=1e-8)
        assert np.allclose(B, b, rtol=0, atol=1e-8)
    else:
        assert np.allclose(A, a, rtol=0, atol=1e-13)
        assert np.allclose(B, b, rtol=0, atol=1e-13)
    assert np.all(A[0] == 1.0) and np.all(B[0] == 1.0)   # no alias at k = 0


def test_printed_forms_for_low_multipoles():
    # eq. 45 as printed (continuum shell averages of y_l^m): with l <= 3 the
    # lattice averages vanish exactly except for l = 0, so
    #   S_000 = Sbar/I + A(b1) + A(b2) + ij-term, A(b) = <dn N* - Sbar C/W^2>_b / I;
    #   S_202: the i = k != j term vanishes and j = k != i is
    #          (5/I) sum_M <y_2^M(k^) [dn N_2^M* - Sbar_2^M C/W^2]>_{b1}
    plan = est.Plan(n=24, box_len=600.0, multipoles=[(0, 0, 0), (2, 0, 2)], n_bins=3, dk=2.5 * 2 * math.pi / 600.0,
                    k_min=0.8 * 2 * math.pi / 600.0, assign_p=3, interlace=True, los="local",
                    observer=(300.0, 300.0, -600.0), box_mode=True)
    from mocks import lognormal_box
    cat = lognormal_box(24, 600.0, 4000, 13, rsd="local", observer=plan.observer)
    res = sn.measure_shot_noise(plan, cat)
    grids, info = est.assign_channels(plan, cat)
    dn = est.spectra(plan, grids)
    nk = sn.n_spectra(plan, cat)
    sb = sn.sbar(plan, cat)
    cw2 = sn.shot_window(plan)
    bg = est.bin_grid(plan)
    ux, uy, uz = est.mode_unit_vectors(plan)
    I = info["I"]
    for b1 in range(3):
        for b2 in range(3):
            sel1 = bg == b1
            a0 = np.mean(dn[(0, 0)][sel1] * np.conj(nk[(0, 0)][sel1]) - sb[(0, 0)] * cw2[sel1]).real / I
            sel2 = bg == b2
            a0b = np.mean(dn[(0, 0)][sel2] * np.conj(nk[(0, 0)][sel2]) - sb[(0, 0)] * cw2[sel2]).real / I
            want = sb[(0, 0)].real / I + a0 + a0b
            got = res["iii"][0, b1, b2] + res["jk"][0, b1, b2] + res["ik"][0, b1, b2]
            assert abs(got - want) <= 1e-10 * (abs(want) + abs(a0) + abs(a0b))
            j2 = 0j
            for M in range(-2, 3):
                y = ang.ylm(2, M, ux[sel1], uy[sel1], uz[sel1])
                j2 += np.mean(y * (dn[(0, 0)][sel1] * np.conj(nk[(2, M)][sel1]) - sb[(2, M)] * cw2[sel1]))
            j2 = (5.0 * j2 / I).real
            assert abs(res["jk"][1, b1, b2] - j2) <= 1e-10 * abs(j2)
            assert abs(res["ik"][1, b1, b2]) <= 1e-10 * abs(j2)
            assert abs(res["iii"][1, b1, b2]) <= 1e-10 * abs(sb[(0, 0)] / I)


def test_sbar_along_the_z_axis():
    # particles straight above the observer: x^ = z, where y_L^M*(z) = delta_M0,
    # so Sbar_L^0 = sum_gal w^3 - alpha^3 sum_ran w^3 and Sbar_L^{M != 0} = 0 (eq. 46)
    plan = est.Plan(n=16, box_len=100.0, multipoles=[(0, 0, 0), (2, 0, 2)], n_bins=2, dk=0.1, los="local",
                    observer=(50.0, 50.0, 0.0), box_mode=False)
    gal = {"pos": np.array([[50.0, 50.0, 10.0], [50.0, 50.0, 30.0], [50.0, 50.0, 70.0]]),
           "w": np.array([1.0, 2.0, 0.5]), "nbar": None}
    ran = {"pos": np.array([[50.0, 50.0, 20.0 + 5 * i] for i in range(7)]), "w": np.full(7, 0.5), "nbar": None}
    alpha = 3.5 / 3.5   # sum_gal w = 3.5, sum_ran w = 3.5
    sb = sn.sbar(plan, gal, ran)
    want = (1.0 + 8.0 + 0.125) - alpha ** 3 * 7 * 0.125
    for L in (0, 2):
        assert abs(sb[(L, 0)] - want) <= 1e-13 * want
        for M in range(1, L + 1):
            assert abs(sb[(L, M)]) <= 1e-13 and abs(sb[(L, -M)]) <= 1e-13


def test_n_spectra_for_particles_on_nodes():
    # NGP without interlacing puts a particle on a node exactly on that node,
    # so W N_L^M(k) is the exact particle sum sum (1, alpha^2) w^2 y_L^M(x^) e^{-ik.x}
    # (eq. 46) away from the Nyquist planes
    plan = est.Plan(n=16, box_len=160.0, multipoles=[(0, 0, 0), (2, 0, 2)], n_bins=2, dk=0.1, assign_p=1,
                    interlace=False, los="local", observer=(80.0, 80.0, -200.0), box_mode=False)
    rng = np.random.default_rng(21)
    nodes = 10.0 * rng.integers(0, 16, size=(15, 3)).astype(np.float64)
    gal = {"pos": nodes[:6], "w": 0.5 + rng.random(6), "nbar": None}
    ran = {"pos": nodes[6:], "w": 0.5 + rng.random(9), "nbar": None}
    alpha = gal["w"].sum() / ran["w"].sum()
    nk = sn.n_spectra(plan, gal, ran)
    W = est.mass_window(plan)
    nx, ny, nz = est.mode_vectors(plan.n)
    keep = (np.abs(nx) < 8) & (np.abs(ny) < 8) & (np.abs(nz) < 8)
    k = plan.k_f * np.stack([nx, ny, nz], axis=-1)
    for (L, M) in [(0, 0), (2, 0), (2, 1), (2, -2)]:
        want = np.zeros(nx.shape, dtype=np.complex128)
        for cat, f in ((gal, 1.0), (ran, alpha ** 2)):
            u = est.los_unit_vectors(cat["pos"], plan.observer)
            y = ang.ylm(L, M, u[:, 0], u[:, 1], u[:, 2])
            for i, x in enumerate(cat["pos"]):
                want += f * cat["w"][i] ** 2 * y[i] * np.exp(-1j * (k @ x))
        assert np.max(np.abs(nk[(L, M)][keep] * W[keep] - want[keep])) <= 1e-12 * np.max(np.abs(want))
