"""GPU parity of the column assignment (box-mode FP32 plans on 32^3 to 256^3
grids): the particles are assigned per 2 x 2 x N column and the column's z
lines transformed before anything is stored, so these tests compare the
measured B with the oracle and with the same plan on the tile assignment
(which stores the grids and runs the z pass separately)."""
import numpy as np
import pytest

from mocks import lognormal_box
from oracle import estimator as est
from tests.gpu_util import box_request, normwise_errors, oracle_plan, pair_mask, report

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1803_02132_amd as tsb  # noqa: E402


def _measure(req, cat):
    plan = tsb.Plan(**req)
    return plan, plan.measure(tsb.catalog_to_device(cat))


def _both_paths(req, cat):
    """B of the column path, of the tile path, and of the oracle."""
    report("case", {k: v for k, v in req.items() if k != "multipoles"}, req["multipoles"], len(cat["pos"]))
    pc, gc = _measure(req, cat)
    pt, gt = _measure(dict(req, assign_tiles=True), cat)
    assert pc.info.assign_columns == 1 and pt.info.assign_columns == 0
    o = est.measure(oracle_plan(**req), cat)
    return gc, gt, o


@pytest.mark.parametrize("interlace", [True, False])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_columns_match_oracle_and_tiles(p, interlace):
    req = box_request(n=32, assign_p=p, interlace=interlace, n_bins=6,
                      multipoles=[(0, 0, 0), (1, 1, 0), (2, 0, 2), (1, 1, 2)])
    cat = lognormal_box(32, 1000.0, 20000, 40 + p, rsd="local", observer=req["observer"])
    gc, gt, o = _both_paths(req, cat)
    mask = pair_mask(req["multipoles"], req["n_bins"])
    e_or = normwise_errors(gc["B"], o["B"], mask)
    e_tl = normwise_errors(gc["B"], gt["B"], mask)
    report("columns vs oracle", e_or, "vs tiles", e_tl)
    assert np.all(e_or <= 1e-4)
    assert np.all(e_tl <= 1e-4)
    assert gc["I"] == pytest.approx(o["I"], rel=1e-12)


@pytest.mark.parametrize("n", [64, 128])
def test_columns_larger_grids(n):
    # several columns per XCD band, the 8 x 16 four-step split at 128
    req = box_request(n=n, n_bins=8, dk=0.012, multipoles=[(0, 0, 0), (2, 0, 2)])
    cat = lognormal_box(n, 1000.0, 60000, 50 + n, rsd="local", observer=req["observer"])
    gc, gt, o = _both_paths(req, cat)
    mask = pair_mask(req["multipoles"], req["n_bins"])
    e_or = normwise_errors(gc["B"], o["B"], mask)
    e_tl = normwise_errors(gc["B"], gt["B"], mask)
    report("columns", n, "vs oracle", e_or, "vs tiles", e_tl)
    assert np.all(e_or <= 1e-4) and np.all(e_tl <= 1e-4)


def test_columns_global_los_one_grid():
    req = box_request(n=32, los="global", multipoles=[(0, 0, 0), (2, 0, 2)], n_bins=6)
    cat = lognormal_box(32, 1000.0, 20000, 61, rsd="global")
    gc, gt, o = _both_paths(req, cat)
    mask = pair_mask(req["multipoles"], req["n_bins"])
    e_or = normwise_errors(gc["B"], o["B"], mask)
    report("columns, global LOS", e_or)
    assert np.all(e_or <= 1e-4)


def test_columns_dense_and_crowded():
    # 200k particles on 32^3 (thousands of visits per column: a coarse column
    # scale) plus 30k in one cell, and positions on and just outside the faces
    rng = np.random.default_rng(62)
    L, h = 1000.0, 1000.0 / 32
    back = rng.random((200000, 3)) * L
    crowd = (np.array([8.0, 15.0, 31.0]) + 0.9 * rng.random((30000, 3))) * h
    edge = np.array([0.0, L, -1e-3, L + 1e-3, np.nextafter(np.float32(L), np.float32(0)), 0.5 * L], np.float32)
    faces = rng.choice(edge, size=(3000, 3))
    cat = {"pos": np.concatenate([back, crowd, faces]).astype(np.float32)}
    req = box_request(n=32, n_bins=6, multipoles=[(0, 0, 0), (2, 0, 2)])
    gc, gt, o = _both_paths(req, cat)
    mask = pair_mask(req["multipoles"], req["n_bins"])
    e_or = normwise_errors(gc["B"], o["B"], mask)
    report("columns, dense + crowded + faces", e_or)
    assert np.all(e_or <= 1e-4)


def test_columns_order_free():
    # fixed-point sums: the shuffled catalogue gives the same bits
    req = box_request(n=64, n_bins=6, dk=0.015)
    cat = lognormal_box(64, 1000.0, 50000, 63, rsd="local", observer=req["observer"])
    perm = np.random.default_rng(3).permutation(len(cat["pos"]))
    plan = tsb.Plan(**req)
    assert plan.info.assign_columns == 1
    a = plan.measure(tsb.catalog_to_device(cat))["B"]
    b = plan.measure(tsb.catalog_to_device({"pos": cat["pos"][perm]}))["B"]
    assert np.array_equal(np.nan_to_num(a), np.nan_to_num(b))


def test_assign_call_still_returns_tile_grids():
    # the grids themselves (tsb_assign) come from the tile path of a column plan
    req = box_request(n=32, multipoles=[(0, 0, 0), (2, 0, 2)])
    cat = lognormal_box(32, 1000.0, 5000, 64, rsd="local", observer=req["observer"])
    plan = tsb.Plan(**req)
    assert plan.info.assign_columns == 1
    grids = plan.assign(tsb.catalog_to_device(cat)).cpu().numpy()
    og, _ = est.assign_channels(oracle_plan(**req), cat)
    for c, (L, M, part) in enumerate(plan.channels()):
        ref = og[(L, M)][0]
        ref = ref.real if part == 0 else ref.imag
        assert np.max(np.abs(grids[0, c] - ref)) <= 4e-6 * max(np.max(np.abs(ref)), 1.0)
    # and a measurement after it runs the column path again
    g = plan.measure(tsb.catalog_to_device(cat))
    o = est.measure(oracle_plan(**req), cat)
    assert np.all(normwise_errors(g["B"], o["B"], pair_mask(req["multipoles"], req["n_bins"])) <= 1e-4)
