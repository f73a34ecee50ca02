"""Pins of the oracle's estimator (no GPU).

Each test checks the oracle against something other than itself: closed forms
of the assignment kernels and their transforms, a direct (non-FFT) Fourier sum,
an independent lattice-point count, the direct triangle sum of eq. 35, the
Legendre special case of Sec. 3.1, and exact invariances of a J = 0 quantity.
"""
import math

import numpy as np
import pytest

from oracle import angular as ang
from oracle import estimator as est
from mocks import lognormal_box


def small_plan(**kw):
    base = dict(n=16, box_len=100.0, multipoles=[(0, 0, 0), (1, 1, 0), (2, 0, 2), (1, 1, 2), (2, 2, 0)],
                n_bins=4, dk=1.5 * 2 * math.pi / 100.0, assign_p=3, interlace=True, los="local",
                observer=(50.0, 50.0, -150.0), box_mode=True)
    base.update(kw)
    return est.Plan(**base)


def small_cat(seed=3, n_target=3000, n=16, box=100.0, rsd="local", observer=(50.0, 50.0, -150.0)):
    return lognormal_box(n, box, n_target, seed, rsd=rsd, observer=observer,
                         pk=lambda k: 2e3 * np.where(k > 0, (np.maximum(k, 1e-9) / 0.1) ** -1.5, 0))


# ----------------------------------------------------------------------------
# assignment


def _kernel_of_distance(s, p):
    """Hockney & Eastwood kernels as functions of the node-particle distance s (grid units)."""
    s = abs(s)
    if p == 1:
        return 1.0 if s < 0.5 else 0.0
    if p == 2:
        return max(0.0, 1.0 - s)
    if s < 0.5:
        return 0.75 - s * s
    if s < 1.5:
        return 0.5 * (1.5 - s) ** 2
    return 0.0


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("shift", [0.0, 0.5])
def test_assignment_conserves_weight(p, shift):
    plan = small_plan(assign_p=p)
    rng = np.random.default_rng(p)
    pos = rng.random((500, 3)) * plan.box_len
    w = rng.random(500) + 0.5
    D = est.assign(pos, w, plan, shift=shift)
    assert abs(D.sum().real - w.sum()) < 1e-12 * w.sum()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_assignment_single_particle_matches_distance_kernel(p):
    plan = small_plan(assign_p=p, n=8, box_len=8.0)
    rng = np.random.default_rng(10 + p)
    for _ in range(20):
        x = rng.random(3) * 8.0
        D = est.assign(x[None, :], np.ones(1), plan).real
        for i in range(8):
            for j in range(8):
                for k in range(8):
                    want = 1.0
                    for a, node in enumerate((i, j, k)):
                        s = x[a] - node
                        s = (s + 4.0) % 8.0 - 4.0          # periodic distance
                        want *= _kernel_of_distance(s, p)
                    assert D[i, j, k] == pytest.approx(want, abs=1e-14)


def test_tsc_node_stencil_and_transform():
    # a particle on a node: 3/4 at the node, 1/8 at each neighbour per axis;
    # its DFT is prod_i (3/4 + cos(2 pi n_i/N)/4) e^{-i k.x}
    plan = small_plan(n=16, box_len=16.0, interlace=False)
    x = np.array([[3.0, 5.0, 7.0]])
    D = est.assign(x, np.ones(1), plan).real
    assert D[3, 5, 7] == pytest.approx(0.75 ** 3, abs=1e-15)
    assert D[2, 5, 7] == pytest.approx(0.125 * 0.75 ** 2, abs=1e-15)
    F = np.fft.fftn(D)
    nx, ny, nz = est.mode_vectors(16)
    th = 2 * math.pi / 16
    want = ((0.75 + 0.25 * np.cos(th * nx)) * (0.75 + 0.25 * np.cos(th * ny)) * (0.75 + 0.25 * np.cos(th * nz))
            * np.exp(-1j * th * (3 * nx + 5 * ny + 7 * nz)))
    assert np.allclose(F, want, atol=1e-13)


def test_spectrum_matches_direct_fourier_sum_at_low_k():
    # deconvolved, interlaced spectrum vs sum_i w_i e^{-ik.x_i}: agreement up to
    # aliasing, small at |n| <= 2 of a 32^3 grid; a wrong interlace phase or
    # deconvolution exponent fails by orders of magnitude
    plan = est.Plan(n=32, box_len=32.0, multipoles=[(0, 0, 0)], n_bins=2, dk=0.1, assign_p=3,
                    interlace=True, los="global", box_mode=False)
    rng = np.random.default_rng(7)
    pos = rng.random((400, 3)) * 32.0
    D1 = est.assign(pos, np.ones(400), plan, 0.0)
    D2 = est.assign(pos, np.ones(400), plan, 0.5)
    spec = est.spectra(plan, {(0, 0): [D1, D2]})[(0, 0)]
    for n in [(1, 0, 0), (0, 2, 1), (1, 1, 1), (2, -1, 0), (-2, 2, 1)]:
        k = 2 * math.pi / 32.0 * np.array(n)
        direct = np.sum(np.exp(-1j * pos @ k))
        got = spec[n[0] % 32, n[1] % 32, n[2] % 32]
        assert abs(got - direct) < 2e-3 * 400 ** 0.5 + 1e-3 * abs(direct)


def _r3_counts(n2max):
    """Number of integer vectors with |n|^2 = s, by an independent enumeration."""
    r3 = np.zeros(n2max + 1, dtype=np.int64)
    lim = int(math.isqrt(n2max))
    for a in range(-lim, lim + 1):
        for b in range(-lim, lim + 1):
            rem = n2max - a * a - b * b
            if rem < 0:
                continue
            for s in range(a * a + b * b, n2max + 1):
                c2 = s - a * a - b * b
                c = math.isqrt(c2)
                if c * c == c2:
                    r3[s] += 1 if c == 0 else 2
    return r3


def test_nmode_against_lattice_point_count():
    plan = est.Plan(n=32, box_len=1000.0, multipoles=[(0, 0, 0)], n_bins=8,
                    dk=2 * 2 * math.pi / 1000.0)
    # shells end at 16 k_f = k_N, so no mode of a shell has a component of N/2 and
    # counting all integer vectors by |n|^2 is the same as counting the grid
    r3 = _r3_counts(16 * 16)
    want = [int(sum(r3[s] for s in range(1, 257) if (2 * b) ** 2 <= s < (2 * b + 2) ** 2))
            for b in range(8)]
    assert list(est.nmode(plan)) == want


# ----------------------------------------------------------------------------
# estimator: FFT route = direct triangle sum, special cases and invariances


def _both_routes(plan, cat, randoms=None):
    grids, info = est.assign_channels(plan, cat, randoms)
    spec = est.spectra(plan, grids)
    Bf, If = est.reduce_fft(plan, spec, info["I"])
    Bb, Ib = est.brute_force(plan, spec, info["I"])
    return Bf, If, Bb, Ib, spec, info


@pytest.mark.parametrize("los", ["local", "global"])
def test_fft_route_equals_triangle_sum_box(los):
    plan = small_plan(los=los, multipoles=[(0, 0, 0), (1, 1, 0), (2, 0, 2), (1, 1, 2), (0, 2, 2)])
    cat = small_cat(rsd="local" if los == "local" else "global")
    Bf, If, Bb, Ib, _, _ = _both_routes(plan, cat)
    for mu in range(len(plan.multipoles)):
        scale = np.nanmax(np.abs(Bb[mu]))
        assert scale > 0
        assert np.nanmax(np.abs(Bf[mu] - Bb[mu])) <= 1e-11 * scale
        # imaginary parts vanish for l1 + l2 + L even
        assert np.nanmax(np.abs(If[mu])) <= 1e-11 * scale


def test_fft_route_equals_triangle_sum_survey_cic_no_interlace():
    plan = small_plan(box_mode=False, assign_p=2, interlace=False, P0=5.0,
                      multipoles=[(0, 0, 0), (2, 0, 2), (4, 0, 4)], observer=(50.0, 50.0, 50.0))
    rng = np.random.default_rng(11)
    centre = np.array([50.0, 50.0, 50.0])

    def shell(npts):
        v = rng.standard_normal((npts, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        r = 20.0 + 25.0 * rng.random(npts) ** (1 / 3)
        return centre + v * r[:, None]

    data = {"pos": shell(1500), "w": 0.5 + rng.random(1500), "nbar": 0.02 + 0.01 * rng.random(1500)}
    rand = {"pos": shell(6000), "w": None, "nbar": 0.02 + 0.01 * rng.random(6000)}
    Bf, If, Bb, Ib, _, info = _both_routes(plan, data, rand)
    assert info["alpha"] > 0
    for mu in range(3):
        scale = np.nanmax(np.abs(Bb[mu]))
        assert np.nanmax(np.abs(Bf[mu] - Bb[mu])) <= 1e-11 * scale


def test_legendre_special_case():
    # Sec. 3.1 / eq. 26: B_{l l 0} = B_l = (2l+1)/I < L_l(k1^.k2^) dn dn dn >, written
    # here as a direct triangle sum with Legendre polynomials (no y, no 3j)
    plan = small_plan(multipoles=[(0, 0, 0), (1, 1, 0), (2, 2, 0)])
    cat = small_cat(seed=5)
    grids, info = est.assign_channels(plan, cat)
    spec = est.spectra(plan, grids)
    Bf, _ = est.reduce_fft(plan, spec, info["I"])
    n = plan.n
    bg = est.bin_grid(plan)
    nx, ny, nz = est.mode_vectors(n)
    d = spec[(0, 0)]
    for b1 in range(plan.n_bins):
        for b2 in range(plan.n_bins):
            s1 = np.nonzero(bg == b1)
            s2 = np.nonzero(bg == b2)
            v1 = np.stack([nx[s1], ny[s1], nz[s1]], 1)
            v2 = np.stack([nx[s2], ny[s2], nz[s2]], 1)
            u1 = v1 / np.linalg.norm(v1, axis=1)[:, None]
            u2 = v2 / np.linalg.norm(v2, axis=1)[:, None]
            mu = u1 @ u2.T
            n3 = np.mod(-(v1[:, None, :] + v2[None, :, :]), n)
            c = d[s1][:, None] * d[s2][None, :] * d[n3[..., 0], n3[..., 1], n3[..., 2]]
            for idx, l in enumerate((0, 1, 2)):
                want = (2 * l + 1) / info["I"] * np.sum(ang.legendre(l, mu) * c).real / (len(v1) * len(v2))
                assert Bf[idx, b1, b2] == pytest.approx(want, rel=1e-10, abs=1e-12 * np.max(np.abs(Bf[idx])))


def test_global_z_quadrupole_special_case():
    # Sec. 4.4: with d = z, B_202 = (5/I) < L_2(k1^.z) dn dn dn >
    plan = small_plan(los="global", multipoles=[(2, 0, 2)])
    cat = small_cat(seed=8, rsd="global")
    grids, info = est.assign_channels(plan, cat)
    spec = est.spectra(plan, grids)
    Bf, _ = est.reduce_fft(plan, spec, info["I"])
    n = plan.n
    bg = est.bin_grid(plan)
    nx, ny, nz = est.mode_vectors(n)
    d = spec[(0, 0)]
    for b1, b2 in [(0, 0), (1, 2), (3, 1), (2, 3)]:
        s1 = np.nonzero(bg == b1)
        s2 = np.nonzero(bg == b2)
        v1 = np.stack([nx[s1], ny[s1], nz[s1]], 1)
        v2 = np.stack([nx[s2], ny[s2], nz[s2]], 1)
        mu1 = v1[:, 2] / np.linalg.norm(v1, axis=1)
        n3 = np.mod(-(v1[:, None, :] + v2[None, :, :]), n)
        c = d[s1][:, None] * d[s2][None, :] * d[n3[..., 0], n3[..., 1], n3[..., 2]]
        want = 5.0 / info["I"] * np.sum(ang.legendre(2, mu1)[:, None] * c).real / (len(v1) * len(v2))
        assert Bf[0, b1, b2] == pytest.approx(want, rel=1e-10)


def _measure_B(plan, cat):
    grids, info = est.assign_channels(plan, cat)
    spec = est.spectra(plan, grids)
    return est.reduce_fft(plan, spec, info["I"])[0]


def test_axis_permutation_invariance():
    # a J = 0 multipole is a rotation scalar: permuting the catalogue axes
    # together with the observer leaves every B unchanged
    plan = small_plan(multipoles=[(0, 0, 0), (2, 0, 2), (1, 1, 2), (2, 2, 0)], observer=(50.0, 40.0, -120.0))
    cat = small_cat(seed=12, observer=(50.0, 40.0, -120.0))
    B0 = _measure_B(plan, cat)
    pos = cat["pos"].astype(np.float64)
    obs = np.array(plan.observer)
    perm = [1, 2, 0]
    plan_p = small_plan(multipoles=plan.multipoles, observer=tuple(obs[perm]))
    Bp = _measure_B(plan_p, {"pos": pos[:, perm]})
    for mu in range(len(plan.multipoles)):
        assert np.max(np.abs(Bp[mu] - B0[mu])) <= 1e-10 * np.max(np.abs(B0[mu]))


def _mirror_x(pos, plane, L):
    out = np.asarray(pos, np.float64).copy()
    out[:, 0] = np.mod(2.0 * plane - out[:, 0], L)
    return out


def test_reflection_invariance_survey_interlaced():
    # parity: mirroring the catalogue (and randoms, observer) in a plane through
    # the observer leaves every l1 + l2 + L even multipole unchanged
    L = 100.0
    mps = [(0, 0, 0), (2, 0, 2), (1, 1, 2), (2, 2, 2)]
    obs = (50.0, 40.0, 45.0)
    plan = small_plan(multipoles=mps, observer=obs, box_mode=False, interlace=True)
    rng = np.random.default_rng(21)
    data = {"pos": 10.0 + 80.0 * rng.random((2500, 3))}
    rand = {"pos": 10.0 + 80.0 * rng.random((10000, 3))}
    g0, i0 = est.assign_channels(plan, data, rand)
    B0 = est.reduce_fft(plan, est.spectra(plan, g0), i0["I"])[0]
    g1, i1 = est.assign_channels(plan, {"pos": _mirror_x(data["pos"], 50.0, L)},
                                 {"pos": _mirror_x(rand["pos"], 50.0, L)})
    B1 = est.reduce_fft(plan, est.spectra(plan, g1), i1["I"])[0]
    for mu in range(len(mps)):
        assert np.max(np.abs(B1[mu] - B0[mu])) <= 1e-10 * np.max(np.abs(B0[mu]))


def test_reflection_invariance_box_node_symmetric_plane():
    # in box mode the node term of R7 uses each node's own LOS, so the mirror must
    # map nodes onto nodes: the plane x = (N-1) H / 2 (first grid only); particles
    # are kept where their mirror image needs no periodic wrap (its LOS would differ)
    L = 100.0
    n = 16
    plane = 0.5 * (n - 1) * L / n
    mps = [(0, 0, 0), (2, 0, 2), (1, 1, 2)]
    obs = (plane, 40.0, -120.0)
    plan = small_plan(multipoles=mps, observer=obs, interlace=False)
    cat = small_cat(seed=12, observer=obs)
    pos = cat["pos"].astype(np.float64)
    pos = pos[pos[:, 0] <= 2.0 * plane]
    B0 = _measure_B(plan, {"pos": pos})
    B1 = _measure_B(plan, {"pos": _mirror_x(pos, plane, L)})
    for mu in range(len(mps)):
        assert np.max(np.abs(B1[mu] - B0[mu])) <= 1e-10 * np.max(np.abs(B0[mu]))


def test_periodic_translation_invariance_global_los():
    plan = small_plan(los="global", multipoles=[(0, 0, 0), (2, 0, 2)])
    cat = small_cat(seed=13, rsd="global")
    B0 = _measure_B(plan, cat)
    h = plan.box_len / plan.n
    shifted = {"pos": np.mod(cat["pos"].astype(np.float64) + np.array([3, 5, 11]) * h, plan.box_len)}
    B1 = _measure_B(plan, shifted)
    assert np.max(np.abs(B1 - B0)) <= 1e-10 * np.max(np.abs(B0))


def test_transpose_symmetry():
    # Sec. 2: B_{l1 l2 L}(k1, k2) = B_{l2 l1 L}(k2, k1)
    plan = small_plan(multipoles=[(2, 0, 2), (0, 2, 2), (1, 1, 2)])
    cat = small_cat(seed=14)
    B = _measure_B(plan, cat)
    assert np.max(np.abs(B[0] - B[1].T)) <= 1e-11 * np.max(np.abs(B[0]))
    assert np.max(np.abs(B[2] - B[2].T)) <= 1e-11 * np.max(np.abs(B[2]))


def test_quadrupole_sum_over_three_axes_vanishes():
    # sum over global LOS x^, y^, z^ of y_2^M*(d) = 0 for every M, so the three
    # global-LOS L = 2 multipoles of any field add up to zero
    mps = [(2, 0, 2), (1, 1, 2), (2, 2, 2)]
    cat = small_cat(seed=15, rsd="global")
    tot = 0
    ref = 0
    for d in [(1.0, 0, 0), (0, 1.0, 0), (0, 0, 1.0)]:
        B = _measure_B(small_plan(los="global", los_dir=d, multipoles=mps), cat)
        tot = tot + B
        ref = max(ref, np.max(np.abs(B)))
    assert np.max(np.abs(tot)) <= 1e-11 * ref


def test_far_observer_matches_global_los():
    mps = [(0, 0, 0), (2, 0, 2), (1, 1, 2)]
    cat = small_cat(seed=16, rsd="global")
    Bg = _measure_B(small_plan(los="global", multipoles=mps), cat)
    Bl = _measure_B(small_plan(los="local", observer=(50.0, 50.0, -1e9), multipoles=mps), cat)
    for mu in range(3):
        assert np.max(np.abs(Bl[mu] - Bg[mu])) <= 1e-6 * np.max(np.abs(Bg[mu]))


def test_box_normalisation():
    plan = small_plan()
    cat = small_cat(seed=17)
    _, info = est.assign_channels(plan, cat)
    n = len(cat["pos"])
    assert info["I"] == pytest.approx(n ** 3 / plan.box_len ** 6, rel=1e-14)


def _node_lattice(n, box, origin=(0.0, 0.0, 0.0)):
    """One unit-weight particle on every grid node (float32 positions that are
    exactly the nodes: box / n is a dyadic fraction here)."""
    j = np.arange(n, dtype=np.float64) * (box / n)
    X, Y, Z = np.meshgrid(j + origin[0], j + origin[1], j + origin[2], indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float32)
    assert np.array_equal(pos.astype(np.float64), np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1))
    return {"pos": pos, "w": None, "nbar": None}


def test_box_mean_term_cancels_a_node_lattice():
    # Reading R7 (box mode subtracts (sum w / N^3) y_L^M*(x^_node) at every
    # node): NGP particles sitting on the nodes give D_L^M(node) = y_L^M*(x^_node)
    # exactly, and the mean is one particle per cell, so every channel, the
    # y-weighted ones of the local LOS included, vanishes before any transform,
    # and with it every multipole. A wrong node position, sign or conjugation
    # in the term leaves the L > 0 channels nonzero.
    plan = small_plan(assign_p=1, interlace=False)
    cat = _node_lattice(plan.n, plan.box_len)
    grids, _ = est.assign_channels(plan, cat)
    for (L, M), per in grids.items():
        assert np.max(np.abs(per[0])) == 0.0, (L, M)
    res = est.measure(plan, cat)
    assert np.all(res["B"] == 0.0)
    # the same lattice one quarter cell off the nodes no longer cancels
    off = {"pos": (cat["pos"] + np.float32(0.25 * plan.box_len / plan.n)).astype(np.float32), "w": None,
           "nbar": None}
    grids_off, _ = est.assign_channels(plan, off)
    assert max(np.max(np.abs(per[0])) for (L, M), per in grids_off.items() if L > 0) > 1e-3


def test_interlacing_phase_covariance_under_half_cell_shift():
    # Reading R5 (grid 2 takes the particles shifted by +H/2 per axis; the
    # combination is (D1 + e^{i pi (nx+ny+nz)/N} D2)/2): shifting every particle
    # by H/2 along (1,1,1) turns grid 1 into grid 2 and grid 2 into grid 1
    # shifted by a whole cell, so the combined field picks up exactly
    # e^{-i pi (nx+ny+nz)/N}. A wrong sign or direction of the phase breaks it.
    plan = small_plan(los="global", multipoles=[(0, 0, 0)], assign_p=3, interlace=True)
    n, box = plan.n, plan.box_len
    h = box / n
    rng = np.random.default_rng(21)
    ticks = rng.integers(0, 1024 * n, size=(2000, 3))          # positions on a 1/1024-cell lattice
    pos = (ticks * (h / 1024)).astype(np.float32)
    shifted = (((ticks + 512) % (1024 * n)) * (h / 1024)).astype(np.float32)
    w = (0.5 + rng.random(2000)).astype(np.float32)
    s1 = est.spectra(plan, est.assign_channels(plan, {"pos": pos, "w": w, "nbar": None})[0])[(0, 0)]
    s2 = est.spectra(plan, est.assign_channels(plan, {"pos": shifted, "w": w, "nbar": None})[0])[(0, 0)]
    nx, ny, nz = est.mode_vectors(n)
    keep = (np.abs(nx) != n // 2) & (np.abs(ny) != n // 2) & (np.abs(nz) != n // 2)
    keep[0, 0, 0] = False
    expect = np.exp(-1j * np.pi * (nx + ny + nz) / n) * s1
    assert np.max(np.abs(s2 - expect)[keep]) <= 1e-12 * np.max(np.abs(s1))
    # the opposite phase convention does not satisfy it
    wrong = np.exp(1j * np.pi * (nx + ny + nz) / n) * s1
    assert np.max(np.abs(s2 - wrong)[keep]) > 1e-3 * np.max(np.abs(s1))


def test_survey_normalisation_of_a_uniform_density():
    # Reading R8 (survey I = v_c sum_j (alpha R_j / v_c)^3, R the gridded
    # randoms): for randoms that fill every node once with weight w (NGP), the
    # mean density n-bar = alpha w / v_c is uniform and eq. 37 gives
    # I = integral of n-bar^3 over the box = n-bar^3 V.
    plan = small_plan(assign_p=1, interlace=False, box_mode=False, multipoles=[(0, 0, 0)], los="global")
    rand = _node_lattice(plan.n, plan.box_len)
    rand["w"] = np.full(len(rand["pos"]), 0.75, dtype=np.float32)
    cat = small_cat(seed=23)
    _, info = est.assign_channels(plan, cat, rand)
    vc = plan.box_len ** 3 / plan.n ** 3
    nbar = info["alpha"] * 0.75 / vc
    assert info["alpha"] == pytest.approx(len(cat["pos"]) / (0.75 * len(rand["pos"])), rel=1e-13)
    assert info["I"] == pytest.approx(nbar ** 3 * plan.box_len ** 3, rel=1e-12)


# ----------------------------------------------------------------------------
# FKP weights (O1), alpha (O2) and the mean |k| of a shell


def test_fkp_weight_hand_values():
    # Sec. 5.2, eq. 54: w = w_c / (1 + nbar P0). With nbar P0 = 1 a weight halves,
    # with nbar P0 = 3 it falls to a quarter, with nbar P0 = 0 it is unchanged.
    P0 = 1024.0   # powers of two keep nbar P0 exact
    w_c = np.array([1.0, 2.0, 0.5, 3.0])
    nbar = np.array([1.0, 3.0, 0.0, 1.0]) / 1024.0
    w = est.fkp_weights(w_c, nbar, P0)
    assert np.array_equal(w, np.array([0.5, 0.5, 0.5, 1.5]))
    # no FKP factor without nbar or with P0 <= 0 (R9)
    assert np.array_equal(est.fkp_weights(w_c, None, P0), w_c)
    assert np.array_equal(est.fkp_weights(w_c, nbar, 0.0), w_c)


def test_alpha_with_fkp_weights():
    # Sec. 4.1 with eq. 54: alpha = sum_gal w_c/(1+nbar P0) / sum_ran w_c/(1+nbar P0).
    # Galaxies: 2 at nbar P0 = 1 (w = 1/2), 1 at nbar P0 = 3 (w = 1/4): sum 5/4.
    # Randoms: 8 at nbar P0 = 1 (w = 1/2), 4 at nbar P0 = 0 (w = 1): sum 8.
    P0 = 64.0
    plan = est.Plan(n=16, box_len=100.0, multipoles=[(0, 0, 0)], n_bins=2, dk=0.1, box_mode=False,
                    los="global", P0=P0, assign_p=1)
    gal = {"pos": np.full((3, 3), 30.0), "w": None, "nbar": np.array([1.0, 1.0, 3.0]) / 64.0}
    ran = {"pos": np.full((12, 3), 60.0), "w": None, "nbar": np.array([1.0] * 8 + [0.0] * 4) / 64.0}
    _, info = est.assign_channels(plan, gal, ran)
    assert info["sum_w"] == 1.25
    assert info["sum_w_ran"] == 8.0
    assert info["alpha"] == 1.25 / 8.0


def test_k_eff_against_sum_of_three_squares():
    # mean |k| over a shell's modes, counted by the number r3(s) of integer
    # vectors with |n|^2 = s (an enumeration independent of the mode grid)
    N, box = 32, 1000.0
    kf = 2 * math.pi / box
    plan = est.Plan(n=N, box_len=box, multipoles=[(0, 0, 0)], n_bins=6, dk=2.5 * kf, k_min=0.7 * kf)
    r3 = _r3_counts(3 * (N // 2) ** 2)
    got = est.k_eff(plan)
    for b in range(6):
        lo, hi = plan.k_min + b * plan.dk, plan.k_min + (b + 1) * plan.dk
        num = den = 0.0
        for s in range(1, len(r3)):
            k = kf * math.sqrt(s)
            if lo <= k < hi and r3[s]:
                num += r3[s] * k
                den += r3[s]
        assert den == est.nmode(plan)[b]
        assert abs(got[b] - num / den) <= 1e-13 * (num / den)


@pytest.mark.slow
def test_fft_route_equals_triangle_sum_c1():
    # the 32^3 box of the smallest configuration: CIC, global z LOS, 8 shells of
    # 2 k_f, {000, 202}, every pair of both multipoles by both routes (eq. 35 vs eq. 41)
    plan = est.Plan(n=32, box_len=1000.0, multipoles=[(0, 0, 0), (2, 0, 2)], n_bins=8,
                    dk=2 * 2 * math.pi / 1000.0, assign_p=2, los="global", box_mode=True)
    cat = lognormal_box(32, 1000.0, 20000, 1, rsd="global")
    grids, info = est.assign_channels(plan, cat)
    spec = est.spectra(plan, grids)
    Bf, If = est.reduce_fft(plan, spec, info["I"])
    Bb, Ib = est.brute_force(plan, spec, info["I"])
    for mu in range(2):
        scale = np.nanmax(np.abs(Bb[mu]))
        assert scale > 0
        assert np.nanmax(np.abs(Bf[mu] - Bb[mu])) <= 1e-12 * scale
        assert np.nanmax(np.abs(If[mu])) <= 1e-12 * scale


# ----------------------------------------------------------------------------
# first-vertex LOS (App. B; reading R12)

X1_MULTIPOLES = [(0, 0, 0), (2, 0, 2), (0, 2, 2), (1, 1, 2), (2, 2, 2), (1, 1, 0)]


def test_first_vertex_fft_route_equals_triangle_sum():
    # eq. 35 with y_L^M*(x^) on the first field's density, summed directly over
    # the shell pairs, against the FFT route with the weighted shell fields
    plan = small_plan(vertex="x1", multipoles=X1_MULTIPOLES)
    cat = small_cat(seed=21)
    Bf, If, Bb, Ib, _, _ = _both_routes(plan, cat)
    for mu in range(len(X1_MULTIPOLES)):
        scale = np.nanmax(np.abs(Bb[mu]))
        assert scale > 0
        assert np.nanmax(np.abs(Bf[mu] - Bb[mu])) <= 1e-11 * scale
        assert np.nanmax(np.abs(If[mu])) <= 1e-11 * scale


def test_first_vertex_equals_third_vertex_at_L0_and_differs_at_L2():
    # y_0^0 = 1 carries no LOS, so L = 0 does not depend on the vertex (App. B);
    # at L = 2 the two vertices give different numbers near the observer
    cat = small_cat(seed=22, observer=(50.0, 50.0, -30.0))
    kw = dict(multipoles=X1_MULTIPOLES, observer=(50.0, 50.0, -30.0))
    B1 = _measure_B(small_plan(vertex="x1", **kw), cat)
    B3 = _measure_B(small_plan(vertex="x3", **kw), cat)
    for mu, (l1, l2, L) in enumerate(X1_MULTIPOLES):
        scale = np.max(np.abs(B3[mu]))
        d = np.max(np.abs(B1[mu] - B3[mu]))
        if L == 0:
            assert d <= 1e-12 * scale
        else:
            assert d >= 1e-3 * scale


def test_first_vertex_far_observer_matches_global_los():
    mps = [(0, 0, 0), (2, 0, 2), (0, 2, 2), (1, 1, 2)]
    cat = small_cat(seed=16, rsd="global")
    Bg = _measure_B(small_plan(los="global", multipoles=mps), cat)
    B1 = _measure_B(small_plan(los="local", vertex="x1", observer=(50.0, 50.0, -1e9), multipoles=mps), cat)
    for mu in range(len(mps)):
        assert np.max(np.abs(B1[mu] - Bg[mu])) <= 1e-6 * np.max(np.abs(Bg[mu]))


# second-vertex LOS (App. B; reading R12 with the weight on the second field)

def test_second_vertex_fft_route_equals_triangle_sum():
    # eq. 35 with y_L^M*(x^) on the second field's density, summed directly
    plan = small_plan(vertex="x2", multipoles=X1_MULTIPOLES)
    cat = small_cat(seed=23)
    Bf, If, Bb, Ib, _, _ = _both_routes(plan, cat)
    for mu in range(len(X1_MULTIPOLES)):
        scale = np.nanmax(np.abs(Bb[mu]))
        assert scale > 0
        assert np.nanmax(np.abs(Bf[mu] - Bb[mu])) <= 1e-11 * scale
        assert np.nanmax(np.abs(If[mu])) <= 1e-11 * scale


def test_second_vertex_is_the_first_with_the_fields_exchanged():
    # 3j(l2 l1 L; m2 m1 M) = (-1)^{l1+l2+L} 3j(l1 l2 L; m1 m2 M), and H_{l1 l2 L}
    # takes the same sign: B^{x2}_{l1 l2 L}(k1, k2) = B^{x1}_{l2 l1 L}(k2, k1)
    obs = (50.0, 50.0, -30.0)
    cat = small_cat(seed=24, observer=obs)
    B1 = _measure_B(small_plan(vertex="x1", multipoles=X1_MULTIPOLES, observer=obs), cat)
    B2 = _measure_B(small_plan(vertex="x2", multipoles=X1_MULTIPOLES, observer=obs), cat)
    for mu, (l1, l2, L) in enumerate(X1_MULTIPOLES):
        nu = X1_MULTIPOLES.index((l2, l1, L))
        scale = np.max(np.abs(B1[nu]))
        assert scale > 0
        assert np.max(np.abs(B2[mu] - B1[nu].T)) <= 1e-12 * scale
    # and it is not the first vertex itself where l1 != l2
    mu = X1_MULTIPOLES.index((2, 0, 2))
    assert np.max(np.abs(B2[mu] - B1[mu])) >= 1e-3 * np.max(np.abs(B1[mu]))


def test_second_vertex_equals_third_vertex_at_L0_and_far_observer_matches_global_los():
    obs = (50.0, 50.0, -30.0)
    cat = small_cat(seed=25, observer=obs)
    B2 = _measure_B(small_plan(vertex="x2", multipoles=X1_MULTIPOLES, observer=obs), cat)
    B3 = _measure_B(small_plan(vertex="x3", multipoles=X1_MULTIPOLES, observer=obs), cat)
    for mu, (l1, l2, L) in enumerate(X1_MULTIPOLES):
        scale = np.max(np.abs(B3[mu]))
        d = np.max(np.abs(B2[mu] - B3[mu]))
        if L == 0:
            assert d <= 1e-12 * scale
        else:
            assert d >= 1e-3 * scale
    mps = [(0, 0, 0), (2, 0, 2), (0, 2, 2), (1, 1, 2)]
    cat = small_cat(seed=16, rsd="global")
    Bg = _measure_B(small_plan(los="global", multipoles=mps), cat)
    B2 = _measure_B(small_plan(los="local", vertex="x2", observer=(50.0, 50.0, -1e9), multipoles=mps), cat)
    for mu in range(len(mps)):
        assert np.max(np.abs(B2[mu] - Bg[mu])) <= 1e-6 * np.max(np.abs(Bg[mu]))
