"""Batched and served measurements through the C ABI.

Every result must equal the plain single-catalogue measurement on the same
inputs bitwise (the kernels are order-independent and each workspace is
private), whether it ran through the captured graph, in a batch of mixed grid
sizes, or on the server alone or in a mix of concurrent requests; one of them
is also checked against the FP64 oracle.
"""

import numpy as np
import pytest

from mocks import lognormal_box
from oracle import estimator as est
from tests.gpu_util import oracle_plan, pair_mask, normwise_errors, box_request, report

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1803_02132_amd as tsb  # noqa: E402


def _say(*a):
    report(*a)


def _same(a, b):
    return np.array_equal(np.nan_to_num(a, nan=7.0), np.nan_to_num(b, nan=7.0))


def _cat(n, seed, n_target):
    return lognormal_box(n, 1000.0, n_target, seed, rsd="local", observer=(500.0, 500.0, -1500.0))


def _requests():
    # three geometries: 32^3, 48^3 (radix 3), 64^3, TSC + interlacing, local LOS, FP32
    return [box_request(n=32, n_bins=6), box_request(n=48, n_bins=6), box_request(n=64, n_bins=6)]


def test_graph_equals_direct_launches():
    req = box_request(n=32, n_bins=6)
    plan_g, plan_d = tsb.Plan(**req), tsb.Plan(**req)
    plan_d.set_graphs(False)
    for k, (seed, n_target) in enumerate([(21, 8000), (22, 30000), (23, 12000)]):
        _say("graph vs direct", seed, n_target)   # the second catalogue regrows the particle buffers
        dev = tsb.catalog_to_device(_cat(32, seed, n_target))
        a = plan_g.measure(dev)["B"]
        b = plan_d.measure(dev)["B"]
        assert _same(a, b), k


def test_batch_of_mixed_grids_matches_single_measurements():
    reqs = _requests()
    plans = [tsb.Plan(**r) for r in reqs]
    items = [(0, 31, 10000), (1, 32, 20000), (2, 33, 40000), (1, 34, 15000), (0, 35, 5000), (2, 36, 25000)]
    devs, single = [], []
    for gi, seed, n_target in items:
        cat = _cat(reqs[gi]["n"], seed, n_target)
        devs.append(tsb.catalog_to_device(cat))
        single.append(plans[gi].measure(devs[-1])["B"])
    _say("batch of", len(items))
    out = tsb.measure_batch([plans[gi] for gi, _, _ in items], devs)
    for k, o in enumerate(out):
        assert _same(o["B"], single[k]), k
    # the radix-3 grid against the oracle
    gi, seed, n_target = items[1]
    o = est.measure(oracle_plan(**reqs[gi]), _cat(reqs[gi]["n"], seed, n_target))
    err = normwise_errors(out[1]["B"], o["B"], pair_mask(reqs[gi]["multipoles"], reqs[gi]["n_bins"]))
    _say("48^3 batch item vs oracle", err)
    assert np.all(err <= 1e-4)


def test_server_alone_and_in_a_mix():
    reqs = _requests()
    tmpl = [tsb.Plan(**r) for r in reqs]
    cats = {k: tsb.catalog_to_device(_cat(reqs[g]["n"], 40 + k, 12000 + 3000 * k)) for k, g in
            enumerate([0, 1, 2, 0, 1])}
    geo = [0, 1, 2, 0, 1]
    srv = tsb.Server(8 << 30, 3)
    try:
        _say("server: alone")
        lat_alone, alone = srv.wait(srv.submit(tmpl[0], cats[0]))
        assert lat_alone > 0
        _say("server: mix")
        tickets = [(k, srv.submit(tmpl[geo[k]], cats[k])) for k in [1, 0, 2, 3, 0, 4, 2]]
        res = [(k, srv.wait(t)) for k, t in tickets]
        for k, (lat, B) in res:
            ref = alone if k == 0 else tmpl[geo[k]].measure(cats[k])["B"]
            assert _same(B, ref), k
            assert lat > 0
        peak, released = srv.stats()
        _say("server mix: peak requests running at once", peak, "workspaces released", released)
        assert peak >= 2   # requests of different geometries overlapped on the device
    finally:
        srv.close()


def test_server_under_a_tight_budget():
    # fewer slots than geometries and a budget that holds about one workspace:
    # idle workspaces are released (LRU) and buffers grow for a larger
    # catalogue of a geometry whose idle workspace is too small; every request
    # finishes with the bits of a plain measurement
    reqs = _requests()
    tmpl = [tsb.Plan(**r) for r in reqs]
    biggest = max(p.info.workspace_bytes for p in tmpl)
    srv = tsb.Server(int(1.5 * biggest) + (64 << 20), 2)
    try:
        order = [(0, 60, 4000), (1, 61, 4000), (2, 62, 4000), (0, 63, 60000), (1, 64, 9000), (0, 65, 3000)]
        cats = [tsb.catalog_to_device(_cat(reqs[g]["n"], s, n)) for g, s, n in order]
        tickets = [srv.submit(tmpl[g], c) for (g, _, _), c in zip(order, cats)]
        _say("tight budget: submitted", len(tickets))
        for (g, _, _), c, t in zip(order, cats, tickets):
            lat, B = srv.wait(t)
            assert _same(B, tmpl[g].measure(c)["B"])
        peak, released = srv.stats()
        _say("tight budget: peak running", peak, "released", released)
        assert released >= 2
    finally:
        srv.close()


def test_server_cancels_queued_requests_at_destroy():
    # requests still queued when the server is destroyed are dropped (their
    # output is never written); the running one finishes with correct bits.
    # One slot: the first request also creates its workspace, so the others
    # are still queued when tsb_server_destroy is called right after submit.
    req = box_request(n=64, n_bins=6)
    plan = tsb.Plan(**req)
    dev = tsb.catalog_to_device(_cat(64, 70, 30000))
    ref = plan.measure(dev)["B"]
    srv = tsb.abi.tsb_server_create(8 << 30, 1)
    outs = [np.full_like(ref, 12345.0) for _ in range(12)]
    cs = tsb._cat_struct(dev)
    for B in outs:
        tsb.abi.tsb_server_submit(srv, plan.handle, cs, None, B.ctypes.data)
    tsb.abi.tsb_server_destroy(srv)
    done = [k for k, B in enumerate(outs) if not np.all(B == 12345.0)]
    _say("destroy with 12 queued: finished", len(done), "cancelled", 12 - len(done))
    assert len(done) < 12
    for k in done:
        assert _same(outs[k], ref), k


def test_server_rejects_what_cannot_fit():
    req = box_request(n=32, n_bins=6)
    plan = tsb.Plan(**req)
    srv = tsb.Server(1 << 20, 2)   # 1 MiB: no workspace fits
    try:
        t = srv.submit(plan, tsb.catalog_to_device(_cat(32, 50, 5000)))
        with pytest.raises(tsb.TsbError) as e:
            srv.wait(t)
        assert e.value.code == tsb.abi.TSB_E_NOMEM
    finally:
        srv.close()


def test_autotune_keeps_results_bitwise():
    # the tuned launch schedule changes how work is split, not the arithmetic
    req = box_request(n=64, n_bins=6)
    dev = tsb.catalog_to_device(_cat(64, 41, 40000))
    plan_a, plan_b = tsb.Plan(**req), tsb.Plan(**req)
    ref = plan_a.measure(dev)["B"]
    choice = plan_b.autotune(dev, reps=2)
    _say("autotune choice", choice)
    assert choice["tile_wgs"] >= 1
    assert choice["reduce_row_tasks"] == -1   # this plan (M = 48) does not run the one-pass reduction
    assert all(v in (8, 16, 32, 64) for k, v in choice.items()
               if k not in ("tile_wgs", "reduce_row_tasks", "reduce_block"))   # 0 (the rule) is not listed
    assert _same(plan_b.measure(dev)["B"], ref)
    plan_b.set_graphs(False)
    assert _same(plan_b.measure(dev)["B"], ref)


@pytest.mark.parametrize("mults,n_bins,dk_kf", [
    ([(0, 0, 0), (2, 0, 2)], 7, 2.0),                                 # kinds in registers, one shell group
    ([(0, 0, 0), (2, 0, 2)], 24, 0.6),                                # kinds in registers, shell groups
    ([(0, 0, 0), (1, 1, 0), (2, 0, 2), (1, 1, 2)], 16, 0.9),          # kind by kind, shell groups
])
def test_reduction_split_and_schedule_reuse_are_bitwise(mults, n_bins, dk_kf):
    # the one-pass reduction's second phase as row tasks, shell tasks or
    # columns transformed once, and a schedule applied from another plan: the
    # same arithmetic, bitwise
    import math
    req = box_request(n=64, n_bins=n_bins, dk=dk_kf * 2.0 * math.pi / 1000.0, multipoles=mults, unfused=2)
    dev = tsb.catalog_to_device(_cat(64, 43, 40000))
    plan = tsb.Plan(**req)
    assert plan.info.fused == 2
    out = {}
    for rt in (0, 1, 2):
        plan.set_schedule({"reduce_row_tasks": rt})
        out[rt] = plan.measure(dev)["B"]
    _say("split", mults, n_bins, "row tasks vs shell tasks vs columns bitwise", _same(out[0], out[1]),
         _same(out[2], out[1]))
    assert _same(out[0], out[1])
    assert _same(out[2], out[1])
    tuned = tsb.Plan(**req)
    choice = tuned.autotune(dev, reps=1)
    other = tsb.Plan(**req)
    other.set_schedule(choice)
    assert _same(other.measure(dev)["B"], out[1])


def test_unfused_reduction_workgroup_size_is_bitwise():
    # the unfused matrix-core reduction in two 512-thread workgroups per CU or
    # one of 1024: the same chunks per workgroup, the same arithmetic
    req = box_request(n=64, n_bins=6, unfused=True)
    dev = tsb.catalog_to_device(_cat(64, 44, 40000))
    plan = tsb.Plan(**req)
    assert plan.info.fused == 0
    out = {}
    for rb in (512, 1024):
        plan.set_schedule({"reduce_block": rb})
        out[rb] = plan.measure(dev)["B"]
    _say("unfused reduction 512 vs 1024 threads bitwise", _same(out[512], out[1024]))
    assert _same(out[512], out[1024])
