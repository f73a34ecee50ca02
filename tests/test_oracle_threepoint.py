"""Pins of the oracle's three-point-function and window multipoles (no GPU).

* The FFT form (eq. 48) against the direct sum over grid points and pairs of
  separation vectors of eq. 47, box and survey, local and global LOS.
* The Legendre form of the L = 0 multipoles (eq. 50).
* A uniform density: Q_000 = 1 in every bin pair (I = nbar^3 V, eq. 37).
* Transpose symmetry zeta_{l1 l2 L}(r1, r2) = zeta_{l2 l1 L}(r2, r1).
"""
import math

import numpy as np
import pytest

from mocks import lognormal_box
from oracle import angular as ang
from oracle import estimator as est
from oracle import threepoint as tp


def _plan(**kw):
    base = dict(n=16, box_len=160.0, multipoles=[(0, 0, 0), (2, 0, 2), (1, 1, 0), (1, 1, 2), (0, 2, 2)],
                n_bins=3, dk=14.0, k_min=8.0, assign_p=3, interlace=True, los="local",
                observer=(80.0, 80.0, -200.0), box_mode=True)
    base.update(kw)
    return est.Plan(**base)


def _spec(plan, seed=2, randoms=None, n_target=3000):
    cat = lognormal_box(plan.n, plan.box_len, n_target, seed, rsd="local", observer=plan.observer,
                        pk=lambda k: 4e3 * np.where(k > 0, (np.maximum(k, 1e-9) / 0.1) ** -1.5, 0))
    grids, info = est.assign_channels(plan, cat, randoms)
    return est.spectra(plan, grids), info


@pytest.mark.parametrize("los", ["local", "global"])
def test_fft_form_equals_the_direct_sum(los):
    plan = _plan(los=los)
    spec, info = _spec(plan)
    z, zi = tp.reduce_fft(plan, spec, info["I"])
    d = tp.direct_sum(plan, spec, info["I"])
    for mu in range(len(plan.multipoles)):
        scale = np.max(np.abs(d[mu]))
        assert scale > 0
        assert np.max(np.abs(z[mu] - d[mu])) <= 1e-11 * scale
        assert np.max(np.abs(zi[mu])) <= 1e-11 * scale   # real for even l1 + l2 + L


def test_fft_form_equals_the_direct_sum_survey_with_zero_separation():
    # bin 0 holds r = 0 (the zero separation, delta_l0), survey mode with FKP
    plan = _plan(box_mode=False, assign_p=2, interlace=False, P0=50.0, k_min=0.0, dk=11.0, n_bins=3,
                 multipoles=[(0, 0, 0), (2, 0, 2), (2, 2, 0)], observer=(80.0, 80.0, 80.0))
    rng = np.random.default_rng(4)
    c = np.array([80.0, 80.0, 80.0])

    def shell(k):
        v = rng.standard_normal((k, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        return c + v * (20.0 + 50.0 * rng.random(k))[:, None]

    data = {"pos": shell(1500), "w": 0.5 + rng.random(1500), "nbar": 0.01 + 0.01 * rng.random(1500)}
    rand = {"pos": shell(6000), "w": None, "nbar": 0.01 + 0.01 * rng.random(6000)}
    grids, info = est.assign_channels(plan, data, rand)
    spec = est.spectra(plan, grids)
    assert tp.n_r(plan)[0] >= 1
    z, _ = tp.reduce_fft(plan, spec, info["I"])
    d = tp.direct_sum(plan, spec, info["I"])
    for mu in range(3):
        assert np.max(np.abs(z[mu] - d[mu])) <= 1e-11 * np.max(np.abs(d[mu]))


def test_legendre_form_of_the_monopoles():
    # eq. 50: zeta_{l l 0} = zeta_l = (2l+1)/I < L_l(r^1 . r^2) dn dn dn >, a direct
    # sum with Legendre polynomials (no y, no 3j)
    plan = _plan(multipoles=[(0, 0, 0), (1, 1, 0), (2, 2, 0)])
    spec, info = _spec(plan, seed=6)
    z, _ = tp.reduce_fft(plan, spec, info["I"])
    n = plan.n
    nx, ny, nz, rb = tp.separation_vectors(plan)
    ux, uy, uz, zero = tp.separation_units(nx, ny, nz)
    d0 = (n ** 3 / plan.volume) * np.fft.ifftn(spec[(0, 0)])
    dv = plan.volume / n ** 3
    # dn(x + H n) for every separation vector of each bin, flattened over x
    shifted = {}
    for b in range(plan.n_bins):
        sel = np.nonzero(rb == b)
        shifted[b] = (np.stack([np.roll(d0, (-a, -bb, -c), axis=(0, 1, 2)).ravel()
                                for a, bb, c in zip(nx[sel], ny[sel], nz[sel])]),
                      np.stack([ux[sel], uy[sel], uz[sel]], axis=1))
    for b1 in range(plan.n_bins):
        for b2 in range(plan.n_bins):
            A, u1 = shifted[b1]
            B, u2 = shifted[b2]
            T = ((A * d0.ravel()[None, :]) @ B.T).real * dv     # v_c sum_x dn(x+r1) dn(x+r2) dn(x)
            cosg = u1 @ u2.T
            for mu, l in enumerate((0, 1, 2)):
                want = (2 * l + 1) / info["I"] * np.sum(ang.legendre(l, cosg) * T) / T.size
                assert abs(z[mu, b1, b2] - want) <= 1e-10 * abs(want) + 1e-14 * np.max(np.abs(z[0]))


def test_window_of_a_uniform_density_is_one():
    # randoms on every node: nbar uniform, I = nbar^3 V (eq. 37), F_0 = G = nbar, so
    # Q_000(r1, r2) = 1 for every pair of bins (the paper's Q_000 -> 1 limit holds
    # everywhere for a uniform window)
    plan = _plan(box_mode=False, multipoles=[(0, 0, 0)], k_min=0.0, dk=9.0, n_bins=4, assign_p=3,
                 interlace=True, observer=(80.0, 80.0, 80.0))
    j = np.arange(16) * 10.0
    X, Y, Z = np.meshgrid(j, j, j, indexing="ij")
    rand = {"pos": np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) + 1e-9, "w": None, "nbar": None}
    data = {"pos": rand["pos"][::7], "w": None, "nbar": None}
    res = tp.measure(plan, data, rand, window=True)
    assert np.allclose(res["zeta"][0], 1.0, rtol=1e-12, atol=0)


def test_transpose_symmetry():
    plan = _plan(multipoles=[(2, 0, 2), (0, 2, 2), (1, 1, 2)])
    spec, info = _spec(plan, seed=9)
    z, _ = tp.reduce_fft(plan, spec, info["I"])
    assert np.allclose(z[0], z[1].T, rtol=1e-11, atol=1e-13 * np.max(np.abs(z[0])))
    assert np.allclose(z[2], z[2].T, rtol=1e-11, atol=1e-13 * np.max(np.abs(z[2])))


def _shot_inputs(plan, seed=7, randoms=None, data=None):
    from oracle import shotnoise as sn
    if data is None:
        data = lognormal_box(plan.n, plan.box_len, 2500, seed, rsd="local", observer=plan.observer,
                             pk=lambda k: 4e3 * np.where(k > 0, (np.maximum(k, 1e-9) / 0.1) ** -1.5, 0))
    grids, info = est.assign_channels(plan, data, randoms)
    spec = est.spectra(plan, grids)
    return spec, sn.n_spectra(plan, data, randoms), sn.sbar(plan, data, randoms), sn.shot_window(plan), info["I"]


@pytest.mark.parametrize("los", ["local", "global"])
def test_shot_noise_is_the_grid_form_of_eq51(los):
    # bins without r = 0: only i = j != k survives (the shell-average analogues
    # Kbar vanish) and only on b1 = b2, where it equals the real-space form of
    # eq. 51 with (-1)^{l1+l2}
    plan = _plan(los=los)
    spec, nk, sb, cw2, I = _shot_inputs(plan)
    out = tp.shot_noise(plan, spec, nk, sb, cw2, I)
    eq51 = tp.shot_noise_eq51(plan, spec, nk, sb, cw2, I)
    for mu in range(len(plan.multipoles)):
        scale = np.nanmax(np.abs(out["ij"][mu]))
        assert scale > 0
        for k in ("iii", "jk", "ik"):
            assert np.max(np.abs(out[k][mu])) <= 1e-12 * scale
        diag = np.eye(plan.n_bins, dtype=bool)
        assert np.max(np.abs(out["ij"][mu][~diag])) <= 1e-12 * scale
        assert np.max(np.abs(out["ij"][mu][diag] - eq51[mu][diag])) <= 1e-11 * scale


def test_shot_noise_zero_separation_bin():
    # a bin holding r = 0: Kbar_0^0 = N^3 / (V N_r) there (the zero separation's
    # y = delta_l0), so the i = j = k term of the monopole is
    # (N H / I) Kbar^2 Sbar_0^0 on that pair
    plan = _plan(k_min=0.0, dk=14.0, multipoles=[(0, 0, 0), (2, 0, 2)])
    spec, nk, sb, cw2, I = _shot_inputs(plan, seed=8)
    out = tp.shot_noise(plan, spec, nk, sb, cw2, I, pairs=[(0, 0), (0, 1)])
    nr = tp.n_r(plan)
    kbar = plan.n ** 3 / (plan.volume * nr[0])
    want = kbar * kbar * sb[(0, 0)].real / I
    assert out["iii"][0, 0, 0] == pytest.approx(want, rel=1e-12)
    assert abs(out["iii"][0, 0, 1]) <= 1e-12 * abs(want)   # bin 1 holds no zero separation


@pytest.mark.parametrize("b", [0, 1])
def test_two_point_sums_in_real_space(b):
    # (1/V) sum_k K(k; b) v(k) = (1/(V N_r)) sum_{n in b} y*(n^) v(Hn) with v the
    # inverse transform of the two-point spectrum (Parseval with the comb of
    # separation vectors; the zero separation of bin 0 enters with y = delta_l0)
    plan = _plan(k_min=0.0, dk=14.0, multipoles=[(0, 0, 0), (2, 0, 2), (1, 1, 0)])
    spec, nk, sb, cw2, I = _shot_inputs(plan, seed=9)
    nx, ny, nz, rb = tp.separation_vectors(plan)
    ux, uy, uz, zero = tp.separation_units(nx, ny, nz)
    sel = rb == b
    assert np.any(zero[sel]) == (b == 0)
    n = plan.n
    got = []
    for (l, m, L, M) in [(0, 0, 0, 0), (2, 1, 2, -1), (2, 0, 2, 0), (1, -1, 2, 1), (0, 0, 2, 2)]:
        v = (n ** 3) * np.fft.ifftn(tp.two_point_spectrum(plan, spec, nk, sb, cw2, L, M))   # sum_k v e^{ik.Hn}
        y = tp.sep_ylm_conj(l, m, ux[sel], uy[sel], uz[sel], zero[sel])
        real = np.sum(y * v[nx[sel] % n, ny[sel] % n, nz[sel] % n]) / (plan.volume * np.sum(sel))
        kspace = tp.two_point_sum(plan, spec, nk, sb, cw2, tp.kernel(plan, l, m, b), L, M)
        got.append((kspace, real))
    scale = max(abs(r) for _, r in got)
    assert scale > 0
    for kspace, real in got:
        assert abs(kspace - real) <= 1e-12 * scale
