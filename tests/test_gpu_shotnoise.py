"""GPU parity of the shot-noise subtraction (Sec. 4.2, eqs. 44-46) through the
C ABI: B - S, the shot noise S and its i = j != k term against the FP64
oracle (oracle/shotnoise.py), box and survey mode, local and global LOS,
FP32 and FP64 plans, and the 128^3 box configuration on every pair against
stored oracle values. Tolerance 1e-4 normwise per multipole for FP32 plans
(each of B - S, S and S_ij against its own largest value), 1e-9 for FP64."""
import math
import os

import numpy as np
import pytest

from mocks import lognormal_box
from mocks.lognormal import WORKLOADS, workload
from oracle import shotnoise as sn
from tests.gpu_util import box_request, oracle_plan, pair_mask, report

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1803_02132_amd as tsb  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _err(got, ref, mask):
    out = []
    for mu in range(ref.shape[0]):
        sel = mask[mu] & np.isfinite(ref[mu])
        scale = np.max(np.abs(ref[mu][sel]))
        out.append(np.max(np.abs(got[mu][sel] - ref[mu][sel])) / scale if scale > 0 else 0.0)
    return np.array(out)


def _check(req, data, randoms=None, tol=1e-4, label=""):
    plan = tsb.Plan(**dict(req, shot_noise=True))
    dd = tsb.catalog_to_device(data)
    dr = None if randoms is None else tsb.catalog_to_device(randoms)
    got = plan.measure(dd, dr)
    S, Sij = plan.shot_noise()
    ref = sn.measure_shot_noise(oracle_plan(**req), data, randoms)
    mask = pair_mask(req["multipoles"], req["n_bins"], req.get("pair_mode", "paper"))
    e_bs = _err(got["B"], ref["B"] - ref["S"], mask)
    e_s = _err(S, ref["S"], mask)
    e_ij = _err(Sij, ref["ij"], mask)
    report(label, "B - S", e_bs, "S", e_s, "S_ij", e_ij)
    assert np.all(e_bs <= tol) and np.all(e_s <= tol) and np.all(e_ij <= tol)
    # the raw estimator of a plain plan is B_out + S
    plain = tsb.Plan(**req).measure(dd, dr)["B"]
    m = np.isfinite(plain)
    assert np.allclose((got["B"] + S)[m], plain[m], rtol=1e-12, atol=1e-12 * np.max(np.abs(plain[m])))
    return got, S


@pytest.mark.parametrize("precision,tol", [("f32", 1e-4), ("f64", 1e-9)])
def test_shot_noise_box_local_los(precision, tol):
    req = box_request(n=32, n_bins=6, multipoles=[(0, 0, 0), (2, 0, 2), (1, 1, 0), (1, 1, 2)], precision=precision)
    cat = lognormal_box(32, 1000.0, 20000, 11, rsd="local", observer=req["observer"])
    _check(req, cat, tol=tol, label=f"box local {precision}")


def test_shot_noise_box_global_los_cic():
    req = box_request(n=32, n_bins=6, los="global", assign_p=2, interlace=False,
                      multipoles=[(0, 0, 0), (2, 0, 2), (2, 2, 0)])
    cat = lognormal_box(32, 1000.0, 30000, 12, rsd="global")
    _check(req, cat, label="box global CIC")


def test_shot_noise_survey_fkp_with_hexadecapole():
    # survey mode: randoms with -alpha in dn, +alpha^2 in N, -alpha^3 in Sbar;
    # l = 4 has non-zero lattice shell averages
    req = box_request(n=32, n_bins=5, box_mode=False, P0=1e4, observer=(500.0, 500.0, 500.0),
                      multipoles=[(0, 0, 0), (2, 0, 2), (4, 0, 4)])
    rng = np.random.default_rng(17)

    def shell(npts):
        v = rng.standard_normal((npts, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        return 500.0 + v * (150.0 + 300.0 * rng.random(npts))[:, None]

    data = {"pos": shell(8000), "w": 0.5 + rng.random(8000), "nbar": 1e-4 * (1 + rng.random(8000))}
    rand = {"pos": shell(30000), "w": None, "nbar": 1e-4 * (1 + rng.random(30000))}
    _check(req, data, rand, label="survey FKP")


def test_shot_noise_box128_every_pair():
    # the 128^3 box configuration (500k particles, TSC + interlacing, local LOS,
    # {000, 110, 202, 112}, 20 shells) against stored oracle values
    exp = np.load(os.path.join(GOLDEN, "box128_shot_seed0.npz"))
    spec, cat = workload("box128", seed=0)
    p = np.asarray(cat["pos"], np.float64)
    assert np.allclose([len(p), p.sum(), (p * p).sum()], exp["checksum"], rtol=1e-12, atol=0)
    w = WORKLOADS["box128"]
    req = dict(n=w["n"], box_len=w["box_len"], multipoles=w["multipoles"], n_bins=w["n_bins"], dk=w["dk"],
               k_min=w["k_min"], assign_p=w["assign_p"], interlace=w["interlace"], los=w["los"],
               observer=w["observer"], box_mode=True, precision="f32", shot_noise=True)
    plan = tsb.Plan(**req)
    got = plan.measure(tsb.catalog_to_device(cat))
    S, Sij = plan.shot_noise()
    mask = pair_mask(req["multipoles"], req["n_bins"])
    e_bs = _err(got["B"], exp["B"] - exp["S"], mask)
    e_s = _err(S, exp["S"], mask)
    e_ij = _err(Sij, exp["S_ij"], mask)
    report("box128 shot noise every pair: B - S", e_bs, "S", e_s, "S_ij", e_ij)
    assert np.all(e_bs <= 1e-4) and np.all(e_s <= 1e-4) and np.all(e_ij <= 1e-4)
