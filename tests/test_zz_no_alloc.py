"""tsb_measure_noalloc against tsb_measure (the entry point it is a variant
of) through the C ABI: bitwise the same B, I and alpha on two calls in a row,
the second with a smaller catalogue, in box and survey mode; results within
the FP32 tolerance of the oracle; a plan too large for the static scratch is
refused with TSB_E_NOMEM and the size it needs."""
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


def _same(a, b):
    return np.array_equal(np.nan_to_num(a, nan=7.0), np.nan_to_num(b, nan=7.0))


def test_noalloc_box_two_calls_second_smaller():
    req = box_request(n=64, n_bins=6)
    plan = tsb.Plan(**req)
    for seed, n_target in ((81, 60000), (82, 9000)):
        cat = lognormal_box(64, 1000.0, n_target, seed, rsd="local", observer=req["observer"])
        dev = tsb.catalog_to_device(cat)
        ref = plan.measure(dev)
        got = plan.measure_noalloc(dev)
        report("noalloc box", seed, len(cat["pos"]), "particles: bitwise", _same(got["B"], ref["B"]))
        assert _same(got["B"], ref["B"])
        assert got["I"] == ref["I"] and got["alpha"] == ref["alpha"]
        o = est.measure(oracle_plan(**req), cat)
        err = normwise_errors(got["B"], o["B"], pair_mask(req["multipoles"], req["n_bins"]))
        report("noalloc box vs oracle", err)
        assert np.all(err <= 1e-4)


def test_noalloc_survey_two_calls_second_smaller():
    req = box_request(n=48, n_bins=5, box_mode=False, P0=1e4, observer=(500.0, 500.0, 500.0),
                      multipoles=[(0, 0, 0), (2, 0, 2), (1, 1, 2)])
    plan = tsb.Plan(**req)
    rng = np.random.default_rng(83)

    def shell(npts):
        v = rng.standard_normal((npts, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        return 500.0 + v * (150.0 + 250.0 * rng.random(npts))[:, None]

    for nd, nr in ((12000, 40000), (3000, 10000)):
        data = {"pos": shell(nd), "w": 0.5 + rng.random(nd), "nbar": 1e-4 * (1 + rng.random(nd))}
        rand = {"pos": shell(nr), "w": None, "nbar": 1e-4 * (1 + rng.random(nr))}
        dd, dr = tsb.catalog_to_device(data), tsb.catalog_to_device(rand)
        ref = plan.measure(dd, dr)
        got = plan.measure_noalloc(dd, dr)
        report("noalloc survey", nd, nr, "bitwise", _same(got["B"], ref["B"]))
        assert _same(got["B"], ref["B"])
        assert got["I"] == ref["I"] and got["alpha"] == ref["alpha"]


def test_noalloc_refuses_a_plan_beyond_the_scratch():
    plan = tsb.Plan(**box_request(n=256, n_bins=20, dk=0.01))
    dev = tsb.catalog_to_device(lognormal_box(64, 1000.0, 5000, 84, rsd="local", observer=(500.0, 500.0, -1500.0)))
    with pytest.raises(tsb.TsbError) as e:
        plan.measure_noalloc(dev)
    report("noalloc refusal:", str(e.value))
    assert e.value.code == tsb.abi.TSB_E_NOMEM and "MiB" in str(e.value)
    # the plan still measures normally afterwards
    assert np.isfinite(plan.measure(dev)["B"]).sum() == plan.info.n_outputs
