"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/triposh.h declares, and its planner (validation, k-shells,
N_mode, reduction grid) agrees with the oracle and the paper's rules."""
import math
import os
import re

import numpy as np
import pytest

import paper_1803_02132_amd as tsb
from oracle import angular as ang
from oracle import estimator as est

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "triposh.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(?:int|const char\*)\s+(tsb_\w+)\s*\(", src)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 10
    lib = tsb.abi._lib
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(tsb.abi.EXPORTED)


def req(**kw):
    base = dict(n=64, box_len=1000.0, multipoles=[(0, 0, 0), (2, 0, 2)], n_bins=8, dk=0.01, k_min=0.0,
                assign_p=3, interlace=True, los="local", observer=(500.0, 500.0, -1000.0))
    base.update(kw)
    return base


@pytest.mark.parametrize("kw", [
    dict(n=32, dk=2 * 2 * math.pi / 1000.0, n_bins=8),
    dict(n=64, dk=0.01, n_bins=10),
    dict(n=48, box_len=700.0, dk=0.013, k_min=0.005, n_bins=7),
    dict(n=128, dk=0.01, n_bins=20),
    dict(n=96, box_len=1500.0, dk=0.008, n_bins=12),
])
def test_nmode_bit_exact_with_oracle(kw):
    r = req(**kw)
    info, nm, ke = tsb.query(**r)
    oplan = est.Plan(n=r["n"], box_len=r["box_len"], multipoles=r["multipoles"], n_bins=r["n_bins"],
                     dk=r["dk"], k_min=r["k_min"])
    assert np.array_equal(nm, est.nmode(oplan))
    # mean |k| of each shell (eq. 38) against the oracle (pinned by a lattice count)
    assert np.allclose(ke, est.k_eff(oplan), rtol=1e-12, atol=0)


def test_explicit_edges_nmode_bit_exact_with_oracle():
    # uneven shells given by their edges (eq. 38 with explicit bins)
    edges = [0.004, 0.011, 0.013, 0.03, 0.0455, 0.071, 0.1]
    r = req(n=64, n_bins=6, edges=edges)
    info, nm, ke = tsb.query(**r)
    oplan = est.Plan(n=64, box_len=1000.0, multipoles=r["multipoles"], n_bins=6, dk=1.0, edges=tuple(edges))
    assert np.array_equal(nm, est.nmode(oplan))
    assert np.allclose(ke, est.k_eff(oplan), rtol=1e-12, atol=0)
    # the same shells as k_min + b dk give the same modes as the equivalent edges
    dk = 0.0125
    a = tsb.query(**req(n=64, n_bins=6, k_min=0.005, dk=dk))[1]
    b = tsb.query(**req(n=64, n_bins=6, edges=[0.005 + i * dk for i in range(7)]))[1]
    assert a.sum() > 0 and np.abs(a - b).sum() <= 2   # edges rounded once vs floor((k - k_min)/dk)


def test_reduction_grid_rule():
    # 256^3, L = 1000, shells to k = 0.2: modes |n| < 31.8, G needs |n| < 63.7,
    # so a 128^3 grid holds every closed triangle without aliasing
    info, _, _ = tsb.query(**req(n=256, n_bins=20, dk=0.01))
    assert (info.n, info.m, info.r_f, info.r_g) == (256, 128, 31, 63)
    assert info.m > 2 * info.r_f + info.r_g
    # shells up to k_N/2 on a small grid: pairs wrap, the full grid is used
    info, _, _ = tsb.query(**req(n=32, n_bins=8, dk=2 * 2 * math.pi / 1000.0))
    assert info.m == 32 and info.r_g == 15


def test_reduction_path_rule():
    # 128^3, {000, 110, 202, 112}, 20 shells: the one-pass reduction would take
    # its shells in groups, so the rule writes the F fields and reduces them on
    # the matrix cores; 256^3 {000, 202} fits one group and stays one-pass
    mults = [(0, 0, 0), (1, 1, 0), (2, 0, 2), (1, 1, 2)]
    r = req(n=128, n_bins=20, dk=0.01, multipoles=mults, interlace=True)
    assert tsb.query(**r)[0].fused == 0
    assert tsb.query(**dict(r, unfused=2))[0].fused == 2
    assert tsb.query(**dict(r, unfused=1))[0].fused == 0
    assert tsb.query(**req(n=256, n_bins=20, dk=0.01, interlace=True))[0].fused == 2
    with pytest.raises(tsb.TsbError) as e:
        tsb.query(**dict(r, unfused=3))
    assert e.value.code == tsb.abi.TSB_E_ARG


def test_column_assignment_rule():
    # box FP32 plans on 32..256 grids with up to four complex grids per copy
    # assign by columns with the z transform; FP64, survey, other sizes and
    # assign_tiles keep the tile assignment
    assert tsb.query(**req(n=64))[0].assign_columns == 1
    assert tsb.query(**req(n=256, n_bins=20, dk=0.01))[0].assign_columns == 1
    assert tsb.query(**req(n=32, los="global", interlace=False, assign_p=1))[0].assign_columns == 1
    assert tsb.query(**req(n=64, precision="f64"))[0].assign_columns == 0
    assert tsb.query(**req(n=64, box_mode=False, P0=1e4))[0].assign_columns == 0
    assert tsb.query(**req(n=48))[0].assign_columns == 0
    assert tsb.query(**req(n=512, box_len=3500.0, n_bins=11, dk=0.02))[0].assign_columns == 0
    assert tsb.query(**req(n=64, assign_tiles=True))[0].assign_columns == 0
    # {000, 202, 404} with a local LOS: 15 channels, 8 grids per copy
    assert tsb.query(**req(n=64, multipoles=[(0, 0, 0), (2, 0, 2), (4, 0, 4)]))[0].assign_columns == 0
    with pytest.raises(tsb.TsbError) as e:
        tsb.query(**req(assign_tiles=2))
    assert e.value.code == tsb.abi.TSB_E_ARG


def test_channel_and_field_counts():
    # local LOS {000, 202}: channels (0,0), (2,0), (2,1)re/im, (2,2)re/im
    info, _, _ = tsb.query(**req())
    assert info.n_channels == 6 and info.n_grids == 3
    # F_0^0, F_2^0 (one packed transform), F_2^1, F_2^2
    assert info.n_fields_f == 6 and info.n_fslots == 3
    # global z LOS {000, 202}: only m = 0 fields survive (Sec. 4.4)
    info, _, _ = tsb.query(**req(los="global"))
    assert info.n_channels == 1 and info.n_fields_f == 2 and info.n_fslots == 1


@pytest.mark.parametrize("pair_mode,count", [("paper", 36 + 64), ("upper", 72), ("diagonal", 16), ("all", 128)])
def test_pair_counts(pair_mode, count):
    info, _, _ = tsb.query(**req(n_bins=8, pair_mode=pair_mode))
    assert info.n_outputs == count


def test_paper_pair_counts_for_eleven_shells():
    # Sec. 5.2: 512^3 in a (3.5 Gpc/h)^3 box, 11 shells of 0.02 h/Mpc give 66 pairs
    # when l1 = l2, else 121
    r = req(n=512, box_len=3500.0, n_bins=11, dk=0.02, k_min=0.0, multipoles=[(0, 0, 0)])
    info, _, _ = tsb.query(**r)
    assert info.n_outputs == 66
    info, _, _ = tsb.query(**dict(r, multipoles=[(2, 0, 2)]))
    assert info.n_outputs == 121


@pytest.mark.parametrize("bad,code", [
    (dict(multipoles=[(1, 0, 0)]), tsb.abi.TSB_E_UNSUPPORTED),      # l1 + l2 + L odd
    (dict(multipoles=[(2, 1, 1)]), tsb.abi.TSB_E_UNSUPPORTED),      # L odd
    (dict(multipoles=[(4, 0, 2)]), tsb.abi.TSB_E_UNSUPPORTED),      # triangle rule
    (dict(multipoles=[(10, 10, 0)]), tsb.abi.TSB_E_UNSUPPORTED),    # l > 8
    (dict(n=20), tsb.abi.TSB_E_UNSUPPORTED),                        # N % 4
    (dict(n=28), tsb.abi.TSB_E_UNSUPPORTED),                        # not 2^a 3^b
    (dict(n_bins=40, dk=0.01), tsb.abi.TSB_E_UNSUPPORTED),          # beyond Nyquist
    (dict(n_bins=0), tsb.abi.TSB_E_ARG),
    (dict(dk=-1.0), tsb.abi.TSB_E_ARG),
    (dict(box_len=0.0), tsb.abi.TSB_E_ARG),
    (dict(assign_p=4), tsb.abi.TSB_E_ARG),
    (dict(los="global", los_dir=(0.0, 0.0, 0.0)), tsb.abi.TSB_E_ARG),
    (dict(box_len=(1000.0, 1000.0, 1200.0)), tsb.abi.TSB_E_UNSUPPORTED),   # one fundamental frequency needed
    (dict(n_bins=2, edges=[0.01, 0.02, 0.02]), tsb.abi.TSB_E_ARG),         # edges not increasing
    (dict(vertex="x2", shot_noise=True), tsb.abi.TSB_E_UNSUPPORTED),       # shot noise: third vertex only
])
def test_invalid_requests(bad, code):
    with pytest.raises(tsb.TsbError) as e:
        tsb.query(**req(**bad))
    assert e.value.code == code
    assert tsb.abi.tsb_last_error()


def test_separation_bins_of_the_3pcf_match_the_oracle():
    # r-bins of the 3PCF and the window multipoles (Sec. 4.3): N_r and the mean
    # |r| of the grid separation vectors per bin, the zero separation included
    from oracle import threepoint as tp
    r = dict(n=16, box_len=160.0, multipoles=[(0, 0, 0), (2, 0, 2)], n_bins=3, dk=11.0, k_min=0.0,
             assign_p=3, interlace=True, box_mode=True)
    for estimator in ("3pcf", "window"):
        info, nr, reff = tsb.query(estimator=estimator, **dict(r, box_mode=estimator == "3pcf"))
        op = est.Plan(**r)
        assert np.array_equal(nr, tp.n_r(op))
        nx, ny, nz, rb = tp.separation_vectors(op)
        dist = 10.0 * np.sqrt(nx * nx + ny * ny + nz * nz)
        for b in range(3):
            assert reff[b] == pytest.approx(np.mean(dist[rb == b]), rel=1e-12)
        assert info.m == 16   # every mode takes part: the reduction grid is the full grid
    assert nr[0] == 7         # r = 0 and the six vectors at r = 10


@pytest.mark.parametrize("bad,code", [
    (dict(estimator="window"), tsb.abi.TSB_E_UNSUPPORTED),                  # window needs randoms
    (dict(estimator="window", shot_noise=True, box_mode=False), tsb.abi.TSB_E_UNSUPPORTED),
    (dict(estimator="3pcf", dk=30.0), tsb.abi.TSB_E_UNSUPPORTED),          # r-bins reach half the box
    (dict(estimator="3pcf", k_min=500.0), tsb.abi.TSB_E_UNSUPPORTED),      # no separation in any bin
    (dict(estimator="3pcf", vertex="x2", k_min=5.0), tsb.abi.TSB_E_UNSUPPORTED),   # LOS at x2: bispectrum only
])
def test_invalid_3pcf_requests(bad, code):
    r = dict(n=16, box_len=160.0, multipoles=[(0, 0, 0)], n_bins=3, dk=11.0, k_min=0.0, box_mode=True)
    r.update(bad)
    with pytest.raises(tsb.TsbError) as e:
        tsb.query(**r)
    assert e.value.code == code


def test_every_table1_multipole_accepted():
    for l1 in range(5):
        for l2 in range(5):
            for L in range(0, 5):
                ok = ang.allowed_multipole(l1, l2, L, require_ordered=False)
                try:
                    tsb.query(**req(multipoles=[(l1, l2, L)]))
                    accepted = True
                except tsb.TsbError:
                    accepted = False
                assert accepted == ok, (l1, l2, L)


def test_single_hip_runtime_in_process():
    # the binding must bind the library to torch's HIP runtime: two runtimes in
    # one process do not share devices
    maps = open("/proc/self/maps").read()
    paths = {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}
    assert len(paths) == 1, paths
