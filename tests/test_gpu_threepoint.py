"""GPU parity of the three-point-function multipoles zeta (Sec. 4.3, eq. 48),
their shot noise (eq. 51) and the window multipoles Q (Sec. 6.1, eq. 58)
through the C ABI, against the FP64 oracle (oracle/threepoint.py): box and
survey mode, local and global LOS, a bin holding the zero separation, FP32 and
FP64 plans. Tolerance 1e-4
normwise per multipole for FP32 plans (the bispectrum's bound: the same
assignment, transforms and reduction, with the separation kernels built in
the plan precision), 1e-9 for FP64."""
import numpy as np
import pytest

from mocks import lognormal_box
from oracle import threepoint as tp
from tests.gpu_util import normwise_errors, oracle_plan, pair_mask, report

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1803_02132_amd as tsb  # noqa: E402

MULTS = [(0, 0, 0), (2, 0, 2), (1, 1, 0), (1, 1, 2), (0, 2, 2), (2, 2, 0)]


def _box(n=32, box_len=320.0, **kw):
    req = dict(n=n, box_len=box_len, multipoles=MULTS, n_bins=4, dk=box_len / n * 2.5, k_min=box_len / n * 1.5,
               assign_p=3, interlace=True, los="local", observer=(box_len / 2, box_len / 2, -1.5 * box_len),
               box_mode=True, precision="f32")
    req.update(kw)
    return req


def _shell_catalogues(centre, r_in, r_out, n_data, n_ran, seed):
    rng = np.random.default_rng(seed)
    c = np.asarray(centre, np.float64)

    def shell(k):
        v = rng.standard_normal((k, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        return c + v * (r_in + (r_out - r_in) * rng.random(k))[:, None]

    # the catalogues hold FP32 values (the library's input type), so that both
    # sides see the same inputs
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    data = {"pos": f32(shell(n_data)), "w": f32(0.5 + rng.random(n_data)), "nbar": f32(1e-3 * (1.0 + rng.random(n_data)))}
    rand = {"pos": f32(shell(n_ran)), "w": None, "nbar": f32(1e-3 * (1.0 + rng.random(n_ran)))}
    return data, rand


def _check(req, data, randoms=None, tol=1e-4, label="", window=False):
    estimator = "window" if window else "3pcf"
    plan = tsb.Plan(**dict(req, estimator=estimator))
    nr_or = tp.n_r(oracle_plan(**req))
    assert np.array_equal(plan.nmode, nr_or)
    got = plan.measure(tsb.catalog_to_device(data), None if randoms is None else tsb.catalog_to_device(randoms))
    ref = tp.measure(oracle_plan(**req), data, randoms, window=window)
    mask = pair_mask(req["multipoles"], req["n_bins"], req.get("pair_mode", "paper"))
    mask &= (nr_or[None, :, None] > 0) & (nr_or[None, None, :] > 0)
    assert np.all(np.isfinite(got["B"][mask]))
    assert np.all(np.isnan(got["B"][~mask]))
    err = normwise_errors(got["B"], ref["zeta"], mask)
    report(label, estimator, "N_r", plan.nmode, "normwise", err, "I", got["I"] / ref["I"] - 1.0)
    assert abs(got["I"] / ref["I"] - 1.0) <= (1e-5 if req.get("precision", "f32") == "f32" else 1e-12)
    assert np.all(err <= tol)
    return got, ref


@pytest.mark.parametrize("precision,tol", [("f32", 1e-4), ("f64", 1e-9)])
def test_zeta_box_local_los(precision, tol):
    req = _box(precision=precision)
    cat = lognormal_box(32, 320.0, 30000, 21, rsd="local", observer=req["observer"])
    _check(req, cat, tol=tol, label=f"box local {precision}")


def test_zeta_box_global_los_cic():
    req = _box(los="global", los_dir=(0.3, -0.2, 1.0), assign_p=2, interlace=False,
               multipoles=[(0, 0, 0), (2, 0, 2), (2, 2, 0), (1, 1, 2)])
    cat = lognormal_box(32, 320.0, 30000, 22, rsd="global")
    _check(req, cat, label="box global CIC")


@pytest.mark.parametrize("precision,tol", [("f32", 1e-4), ("f64", 1e-9)])
def test_zeta_survey_fkp_with_zero_separation(precision, tol):
    # bin 0 holds r = 0 (its y_l^m is delta_l0); FKP weights; randoms with -alpha
    req = _box(box_mode=False, P0=2000.0, observer=(160.0, 160.0, 160.0), k_min=0.0, dk=22.0, n_bins=4,
               precision=precision, assign_p=2, interlace=False,
               multipoles=[(0, 0, 0), (2, 0, 2), (2, 2, 0), (1, 1, 0)])
    data, rand = _shell_catalogues((160.0, 160.0, 160.0), 40.0, 140.0, 20000, 80000, 23)
    _check(req, data, rand, tol=tol, label=f"survey FKP r=0 {precision}")


@pytest.mark.parametrize("precision,tol", [("f32", 1e-4), ("f64", 1e-9)])
def test_window_multipoles(precision, tol):
    req = _box(box_mode=False, P0=2000.0, observer=(160.0, 160.0, 160.0), k_min=0.0, dk=22.0, n_bins=4,
               precision=precision, multipoles=[(0, 0, 0), (2, 0, 2), (0, 2, 2), (2, 2, 0), (1, 1, 2)])
    data, rand = _shell_catalogues((160.0, 160.0, 160.0), 40.0, 140.0, 20000, 80000, 24)
    _check(req, data, rand, tol=tol, label=f"window {precision}", window=True)


def test_zeta_64_grid_several_tiles_edges_every_pair():
    # a 64^3 grid (several assignment tiles, the reduction over 64^3 cells),
    # explicit r edges, every pair
    edges = [5.0, 14.0, 23.0, 35.0, 50.0, 70.0, 95.0]
    req = _box(n=64, box_len=640.0, edges=edges, n_bins=len(edges) - 1, pair_mode="all",
               multipoles=[(0, 0, 0), (1, 1, 0), (2, 0, 2), (2, 2, 2)])
    cat = lognormal_box(64, 640.0, 150000, 25, rsd="local", observer=req["observer"])
    _check(req, cat, label="box 64 edges all pairs")


def test_window_does_not_depend_on_the_galaxy_positions():
    # Q is built from the randoms alone; the galaxies only fix alpha through
    # their weights (Sec. 6.1)
    req = _box(box_mode=False, observer=(160.0, 160.0, 160.0), k_min=0.0, dk=22.0, n_bins=3,
               multipoles=[(0, 0, 0), (2, 0, 2)], precision="f64")
    data, rand = _shell_catalogues((160.0, 160.0, 160.0), 40.0, 140.0, 5000, 20000, 26)
    moved = dict(data, pos=_shell_catalogues((160.0, 160.0, 160.0), 20.0, 100.0, 5000, 1, 27)[0]["pos"])
    p = tsb.Plan(**dict(req, estimator="window"))
    a = p.measure(tsb.catalog_to_device(data), tsb.catalog_to_device(rand))
    b = p.measure(tsb.catalog_to_device(moved), tsb.catalog_to_device(rand))
    m = np.isfinite(a["B"])
    assert np.allclose(a["B"][m], b["B"][m], rtol=1e-12, atol=1e-12 * np.max(np.abs(a["B"][m])))
    assert a["alpha"] == b["alpha"]


def test_masked_model_from_measured_window():
    # Sec. 6.2 end to end: window multipoles Q measured on the GPU (every r-bin
    # pair), then the masked zeta of eqs. 63-64 on the host through the C ABI,
    # against the oracle's masked model on the oracle's Q
    from oracle import masked as mk
    mults = [(0, 0, 0), (1, 1, 0), (2, 2, 0), (2, 0, 2)]
    req = _box(box_mode=False, P0=2000.0, observer=(160.0, 160.0, 160.0), k_min=5.0, dk=20.0, n_bins=4,
               precision="f32", multipoles=mults, pair_mode="all")
    data, rand = _shell_catalogues((160.0, 160.0, 160.0), 40.0, 140.0, 20000, 80000, 28)
    plan = tsb.Plan(**dict(req, estimator="window"))
    Qg = plan.measure(tsb.catalog_to_device(data), tsb.catalog_to_device(rand))["B"]
    Qo = tp.measure(oracle_plan(**req), data, rand, window=True)["zeta"]
    r = np.asarray(plan.k_eff)                       # mean separation per r-bin
    w = np.full(r.size, req["dk"])
    rng = np.random.default_rng(29)
    model = {m: rng.standard_normal((r.size, r.size)) for m in mults}
    got, zb = tsb.masked_zeta(mults, mults, model, mults, {m: Qg[i] for i, m in enumerate(mults)}, r, w)
    want, zb_o = mk.masked_zeta(mults, mults, model, mults, {m: Qo[i] for i, m in enumerate(mults)}, r, w)
    errs = np.array([np.max(np.abs(got[m] - want[m])) / np.max(np.abs(want[m])) for m in mults])
    report("masked model from the measured window: normwise", errs, "zeta_bar", zb, zb_o)
    assert np.all(errs <= 1e-4)
    assert zb == pytest.approx(zb_o, rel=1e-4)



@pytest.mark.parametrize("precision,tol", [("f32", 1e-4), ("f64", 1e-9)])
def test_zeta_shot_noise_box(precision, tol):
    # eq. 51 on the grid: zeta - S, S (the i = j != k term, on b1 = b2 only)
    req = _box(precision=precision, pair_mode="all")
    cat = lognormal_box(32, 320.0, 30000, 32, rsd="local", observer=req["observer"])
    plan = tsb.Plan(**dict(req, estimator="3pcf", shot_noise=True))
    got = plan.measure(tsb.catalog_to_device(cat))
    S, Sij = plan.shot_noise()
    ref = tp.measure_shot_noise(oracle_plan(**req), cat)
    mask = pair_mask(req["multipoles"], req["n_bins"], "all")
    e1 = normwise_errors(got["B"], ref["zeta"] - ref["S"], mask)
    e2 = normwise_errors(S, ref["S"], mask)
    report("3pcf shot noise", precision, "zeta - S", e1, "S", e2)
    assert np.all(e1 <= tol) and np.all(e2 <= tol)
    off = ~np.eye(req["n_bins"], dtype=bool)
    for mu in range(len(req["multipoles"])):
        assert np.max(np.abs(S[mu][off])) <= 1e-6 * np.max(np.abs(S[mu]))


@pytest.mark.parametrize("precision,tol", [("f32", 1e-4), ("f64", 1e-9)])
def test_zeta_shot_noise_with_the_zero_separation_bin(precision, tol):
    # a bin holding r = 0: Kbar_0^0 = N^3/(V N_r) there, so the i = j = k term and
    # the two-point sums (j = k, i = k) join the i = j != k term on its pairs
    req = _box(precision=precision, pair_mode="all", k_min=0.0, dk=25.0, n_bins=3)
    cat = lognormal_box(32, 320.0, 30000, 34, rsd="local", observer=req["observer"])
    plan = tsb.Plan(**dict(req, estimator="3pcf", shot_noise=True))
    got = plan.measure(tsb.catalog_to_device(cat))
    S, Sij = plan.shot_noise()
    ref = tp.measure_shot_noise(oracle_plan(**req), cat)
    mask = pair_mask(req["multipoles"], req["n_bins"], "all")
    e1 = normwise_errors(got["B"], ref["zeta"] - ref["S"], mask)
    e2 = normwise_errors(S, ref["S"], mask)
    e3 = normwise_errors(Sij, ref["ij"], mask)
    report("3pcf shot noise, zero-separation bin", precision, "zeta - S", e1, "S", e2, "S_ij", e3)
    assert np.all(e1 <= tol) and np.all(e2 <= tol) and np.all(e3 <= tol)
    # the other terms are not zero on the zero bin's row and column
    other = ref["S"] - ref["ij"]
    assert np.max(np.abs(other[0][0, :])) > 1e-3 * np.max(np.abs(ref["S"][0]))


@pytest.mark.parametrize("k_min", [8.0, 0.0])   # 0: the first bin holds the zero separation
def test_zeta_shot_noise_survey_global_los(k_min):
    req = _box(box_mode=False, P0=2000.0, observer=(160.0, 160.0, 160.0), los="global", los_dir=(0.2, 0.1, 1.0),
               k_min=k_min, dk=20.0, n_bins=4, pair_mode="all", multipoles=[(0, 0, 0), (2, 0, 2), (1, 1, 0)])
    data, rand = _shell_catalogues((160.0, 160.0, 160.0), 40.0, 140.0, 20000, 80000, 33)
    plan = tsb.Plan(**dict(req, estimator="3pcf", shot_noise=True))
    got = plan.measure(tsb.catalog_to_device(data), tsb.catalog_to_device(rand))
    S, _ = plan.shot_noise()
    ref = tp.measure_shot_noise(oracle_plan(**req), data, rand)
    mask = pair_mask(req["multipoles"], req["n_bins"], "all")
    e1 = normwise_errors(got["B"], ref["zeta"] - ref["S"], mask)
    e2 = normwise_errors(S, ref["S"], mask)
    report("3pcf shot noise survey, r_min", k_min, "zeta - S", e1, "S", e2)
    assert np.all(e1 <= 1e-4) and np.all(e2 <= 1e-4)
