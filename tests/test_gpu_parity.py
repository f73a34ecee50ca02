"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs. Small grids span several tiles and ragged line blocks.

Tolerances: FP64 plans agree to 1e-9 (normwise per multipole); FP32 plans to
1e-4 normwise per multipole (max |dB| / max |B| over the computed pairs). A
node lattice, where the box-mode node term cancels every channel exactly,
leaves B below 1e-6 of the B of a uniform catalogue of the same size.
Assignment grids: FP64 to 1e-12 of the largest value, FP32 node by node to
the fixed-point error model;
N_mode bit-exact.
"""
import math

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


def small_cat(n=32, box_len=1000.0, n_target=20000, seed=1, rsd="local", observer=(500.0, 500.0, -1500.0)):
    return lognormal_box(n, box_len, n_target, seed, rsd=rsd, observer=observer)


def survey_inputs(n=32, box_len=1000.0, seed=4):
    rng = np.random.default_rng(seed)
    centre = np.full(3, box_len / 2)

    def shell(npts):
        v = rng.standard_normal((npts, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        r = 0.2 * box_len + 0.25 * box_len * rng.random(npts) ** (1 / 3)
        return (centre + v * r[:, None]).astype(np.float32)

    data = {"pos": shell(8000), "w": (0.5 + rng.random(8000)).astype(np.float32),
            "nbar": (2e-4 + 1e-4 * rng.random(8000)).astype(np.float32)}
    rand = {"pos": shell(30000), "w": None, "nbar": (2e-4 + 1e-4 * rng.random(30000)).astype(np.float32)}
    return data, rand


def run_both(req, data, rand=None):
    _say("case", {k: v for k, v in req.items() if k != "multipoles"}, req["multipoles"])
    plan = tsb.Plan(**req)
    dd = tsb.catalog_to_device(data)
    rd = tsb.catalog_to_device(rand) if rand is not None else None
    g = plan.measure(dd, rd)
    o = est.measure(oracle_plan(**req), data, rand)
    return plan, g, o


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_assignment_grids(p, precision):
    req = box_request(n=32, multipoles=[(0, 0, 0), (2, 0, 2)], assign_p=p, precision=precision)
    _say("assign", p, precision)
    cat = small_cat()
    plan = tsb.Plan(**req)
    grids = plan.assign(tsb.catalog_to_device(cat)).cpu().numpy()
    op = oracle_plan(**req)
    og, _ = est.assign_channels(op, cat)
    if precision == "f32":
        _fp32_assignment_model(plan, op, cat, grids, og)
        return
    for c, (L, M, part) in enumerate(plan.channels()):
        for copy in range(2):
            ref = og[(L, M)][copy]
            ref = ref.real if part == 0 else ref.imag
            scale = max(np.max(np.abs(ref)), 1.0)
            err = np.max(np.abs(grids[copy, c] - ref))
            assert err <= 1e-12 * scale, (L, M, part, copy, err, scale)


def _fp32_assignment_model(plan, op, cat, grids, og):
    # Error model of FP32 assignment, node by node: FP32 rounding of the summed
    # grid and of the grid after the box-mode mean term, plus, per contribution
    # to a node, the FP32 product c W 2^e (three roundings) rounded to a
    # fixed-point step of at most 2^-22 max|c| (a packed work item of up to 512
    # TSC visits: 512 x 0.42 < 2^8 leaves 22 fraction bits of a 31-bit word;
    # here max|c| = 1): below 2^-21 per contribution. Split tiles add their
    # parts exactly at the plan-wide scale, so the model holds for them too.
    n, p = op.n, op.assign_p
    pos = np.asarray(cat["pos"], np.float64)
    mean = len(pos) / n ** 3
    worst = 0.0
    for copy in range(grids.shape[0]):
        u = est.grid_coordinate(pos, op) + 0.5 * copy
        idx = [est.axis_stencil(u[:, a], p)[0] % n for a in range(3)]
        contrib = np.zeros((n, n, n))
        for a in range(p):
            for b in range(p):
                for c in range(p):
                    np.add.at(contrib, (idx[0][:, a], idx[1][:, b], idx[2][:, c]), 1.0)
        for ch, (L, M, part) in enumerate(plan.channels()):
            ref = og[(L, M)][copy]
            ref = ref.real if part == 0 else ref.imag
            bound = 2.0 ** -22 * (np.abs(ref) + mean) + contrib * 2.0 ** -21
            err = np.abs(grids[copy, ch] - ref)
            assert np.all(err <= bound), (L, M, part, copy, float(np.max(err / bound)))
            worst = max(worst, float(np.max(err)) / max(float(np.max(np.abs(ref))), 1.0))
    _say("fp32 assignment: max error / max(largest value, 1) =", worst)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_assignment_grids_sparse_fp32(p):
    # Few particles per tile: FP32 tiles that run as one work item add the two
    # channels of a complex grid into one 64-bit word at a per-tile scale
    req = box_request(n=32, multipoles=[(0, 0, 0), (2, 0, 2)], assign_p=p, precision="f32")
    _say("assign sparse", p)
    cat = small_cat(n_target=1500, seed=5)
    plan = tsb.Plan(**req)
    grids = plan.assign(tsb.catalog_to_device(cat)).cpu().numpy()
    op = oracle_plan(**req)
    og, _ = est.assign_channels(op, cat)
    _fp32_assignment_model(plan, op, cat, grids, og)


def test_assignment_survey_and_nmode():
    req = box_request(n=32, box_mode=False, P0=1e4, interlace=False, observer=(500.0, 500.0, 500.0),
                      multipoles=[(0, 0, 0), (2, 0, 2)], precision="f64")
    data, rand = survey_inputs()
    plan = tsb.Plan(**req)
    grids = plan.assign(tsb.catalog_to_device(data), tsb.catalog_to_device(rand)).cpu().numpy()
    og, _ = est.assign_channels(oracle_plan(**req), data, rand)
    for c, (L, M, part) in enumerate(plan.channels()):
        ref = og[(L, M)][0]
        ref = ref.real if part == 0 else ref.imag
        assert np.max(np.abs(grids[0, c] - ref)) <= 1e-12 * max(np.max(np.abs(ref)), 1.0)
    assert np.array_equal(np.array(plan.nmode), est.nmode(oracle_plan(**req)))


def test_box32_fp64_global_los():
    # 32^3 box, 20k particles, CIC, plane-parallel LOS along z, {000, 202}, 8 bins of 2 k_f, FP64
    req = box_request(n=32, assign_p=2, interlace=False, los="global", precision="f64", pair_mode="upper")
    cat = small_cat(rsd="global")
    plan, g, o = run_both(req, cat)
    mask = pair_mask(req["multipoles"], req["n_bins"], "upper")
    err = normwise_errors(g["B"], o["B"], mask)
    _say("box32 f64 errors", err)
    assert np.all(np.isnan(g["B"][~mask]))
    assert g["I"] == pytest.approx(o["I"], rel=1e-12)
    assert np.all(err <= 1e-9)


@pytest.mark.parametrize("unfused", [False, True])
@pytest.mark.parametrize("precision,tol", [("f32", 1e-4), ("f64", 1e-9)])
def test_local_los_tsc_interlaced(precision, tol, unfused):
    req = box_request(n=32, multipoles=[(0, 0, 0), (1, 1, 0), (2, 0, 2), (1, 1, 2), (2, 2, 0)],
                      precision=precision, n_bins=6, unfused=unfused)
    cat = small_cat(seed=2)
    plan, g, o = run_both(req, cat)
    mask = pair_mask(req["multipoles"], req["n_bins"])
    err = normwise_errors(g["B"], o["B"], mask)
    _say("local", precision, "unfused" if unfused else "fused", "errors", err)
    assert np.all(err <= tol)


@pytest.mark.parametrize("pair_mode", ["diagonal", "all"])
def test_pair_modes(pair_mode):
    # the diagonal measurement (k1 = k2 only, the cheaper one of Sec. 4.4) and
    # every ordered pair: the computed pairs match the oracle, the others are NaN
    req = box_request(n=32, multipoles=[(0, 0, 0), (1, 1, 0), (2, 0, 2), (1, 1, 2)], precision="f32", n_bins=6,
                      pair_mode=pair_mode)
    cat = small_cat(seed=4)
    plan, g, o = run_both(req, cat)
    mask = pair_mask(req["multipoles"], req["n_bins"], pair_mode)
    err = normwise_errors(g["B"], o["B"], mask)
    _say(pair_mode, "errors", err)
    assert np.all(np.isnan(g["B"][~mask]))
    assert np.all(np.isfinite(g["B"][mask]))
    assert np.all(err <= 1e-4)


def test_survey_fkp():
    req = box_request(n=32, box_mode=False, P0=1e4, interlace=True, observer=(500.0, 500.0, 500.0),
                      multipoles=[(0, 0, 0), (2, 0, 2), (4, 0, 4)], precision="f32", n_bins=6)
    data, rand = survey_inputs()
    plan, g, o = run_both(req, data, rand)
    mask = pair_mask(req["multipoles"], req["n_bins"])
    err = normwise_errors(g["B"], o["B"], mask)
    _say("survey errors", err, "alpha", g["alpha"], o["alpha"], "I", g["I"], o["I"])
    assert g["alpha"] == pytest.approx(o["alpha"], rel=1e-12)
    assert g["I"] == pytest.approx(o["I"], rel=1e-9)
    assert np.all(err <= 1e-4)


X1_MULTS = [(0, 0, 0), (2, 0, 2), (0, 2, 2), (1, 1, 2), (2, 2, 2), (1, 1, 0)]


@pytest.mark.parametrize("vertex", ["x1", "x2"])
@pytest.mark.parametrize("precision,tol", [("f32", 1e-4), ("f64", 1e-9)])
def test_first_vertex_los_box(precision, tol, vertex):
    # App. B: the y_L^M* weight on the first (second) shell field (grid spectra
    # of every channel as sources, packed real channels split by Hermitian
    # symmetry, m < 0 harmonics), G_0^0 only; the observer near the box
    req = box_request(n=32, n_bins=6, vertex=vertex, multipoles=X1_MULTS, precision=precision,
                      observer=(500.0, 400.0, -300.0))
    cat = small_cat(seed=31, observer=(500.0, 400.0, -300.0))
    plan, g, o = run_both(req, cat)
    mask = pair_mask(req["multipoles"], req["n_bins"])
    err = normwise_errors(g["B"], o["B"], mask)
    # and it is a different estimator from the third-vertex one at L > 0
    b3 = tsb.Plan(**dict(req, vertex="x3")).measure(tsb.catalog_to_device(cat))["B"]
    diff = normwise_errors(b3, o["B"], mask)
    _say(vertex, "vertex", precision, "errors", err, "x3 vs its oracle", diff)
    assert np.all(err <= tol)
    assert all(diff[mu] > 1e-3 for mu, m in enumerate(X1_MULTS) if m[2] > 0)


@pytest.mark.parametrize("vertex", ["x1", "x2"])
def test_first_vertex_los_survey_with_hexadecapole(vertex):
    req = box_request(n=32, box_mode=False, P0=1e4, interlace=True, observer=(500.0, 500.0, 500.0), vertex=vertex,
                      multipoles=[(0, 0, 0), (2, 0, 2), (4, 0, 4), (2, 2, 4)], precision="f32", n_bins=6)
    data, rand = survey_inputs()
    plan, g, o = run_both(req, data, rand)
    mask = pair_mask(req["multipoles"], req["n_bins"])
    err = normwise_errors(g["B"], o["B"], mask)
    _say(vertex, "vertex survey errors", err)
    assert np.all(err <= 1e-4)


def test_reduced_grid_matches_full_grid_oracle():
    # shells up to |n| < 8 on a 64^3 grid: the sum over cells runs on M = 32 < N
    req = box_request(n=64, box_len=1000.0, n_bins=4, dk=2.0 * 2.0 * math.pi / 1000.0,
                      multipoles=[(0, 0, 0), (2, 0, 2), (1, 1, 2)], precision="f64")
    info, _, _ = tsb.query(**req)
    assert info.m < info.n
    cat = small_cat(n=64, n_target=60000, seed=3)
    plan, g, o = run_both(req, cat)
    mask = pair_mask(req["multipoles"], req["n_bins"])
    err = normwise_errors(g["B"], o["B"], mask)
    _say("reduced grid M", info.m, "errors", err)
    assert np.all(err <= 1e-9)


def test_bitwise_reproducible():
    req = box_request(n=32, precision="f32")
    cat = small_cat(seed=5)
    plan = tsb.Plan(**req)
    dd = tsb.catalog_to_device(cat)
    a = plan.measure(dd)["B"]
    b = plan.measure(dd)["B"]
    assert np.array_equal(np.nan_to_num(a, nan=7.0), np.nan_to_num(b, nan=7.0))


def test_bad_input_is_reported():
    req = box_request(n=32)
    cat = small_cat(seed=6)
    pos = cat["pos"].copy()
    pos[10, 1] = np.nan
    plan = tsb.Plan(**req)
    with pytest.raises(tsb.TsbError) as e:
        plan.measure(tsb.catalog_to_device({"pos": pos}))
    assert e.value.code == tsb.abi.TSB_E_INPUT


def test_empty_catalogue_is_reported():
    # no particles: the normalisation I vanishes and eq. 41 is undefined; the
    # grids of the assignment are all zero
    req = box_request(n=32, precision="f32")
    plan = tsb.Plan(**req)
    empty = tsb.catalog_to_device({"pos": np.zeros((0, 3), np.float32)})
    with pytest.raises(tsb.TsbError) as e:
        plan.measure(empty)
    assert e.value.code == tsb.abi.TSB_E_INPUT
    assert not np.any(plan.assign(empty).cpu().numpy())
    # the plan still measures a catalogue afterwards
    cat = small_cat(seed=8)
    g = plan.measure(tsb.catalog_to_device(cat))
    o = est.measure(oracle_plan(**req), cat)
    mask = pair_mask(req["multipoles"], req["n_bins"])
    assert np.all(normwise_errors(g["B"], o["B"], mask) <= 1e-4)


def test_single_particle():
    # the smallest catalogue: one particle off the nodes. Only the monopole is
    # compared: with one particle the l > 0 shell sums nearly cancel (the
    # grid's cubic symmetry), leaving values at the rounding level
    req = box_request(n=32, precision="f32", multipoles=[(0, 0, 0)])
    cat = {"pos": np.array([[123.4, 567.8, 901.2]], np.float32)}
    plan, g, o = run_both(req, cat)
    mask = pair_mask(req["multipoles"], req["n_bins"])
    err = normwise_errors(g["B"], o["B"], mask)
    _say("single particle errors", err, "I", g["I"], o["I"])
    assert g["I"] == pytest.approx(o["I"], rel=1e-12)
    assert np.all(err <= 1e-4)


def _assign_vs_oracle(req, cat, tol):
    plan = tsb.Plan(**req)
    grids = plan.assign(tsb.catalog_to_device(cat)).cpu().numpy()
    og, _ = est.assign_channels(oracle_plan(**req), cat)
    for c, (L, M, part) in enumerate(plan.channels()):
        for copy in range(grids.shape[0]):
            ref = og[(L, M)][copy]
            ref = ref.real if part == 0 else ref.imag
            scale = max(np.max(np.abs(ref)), 1.0)
            err = np.max(np.abs(grids[copy, c] - ref))
            assert err <= tol * scale, (L, M, part, copy, err, scale)
    return grids


def test_assignment_order_independent():
    # the catalogue in cell order (as generated) and shuffled give identical bits
    req = box_request(n=32, precision="f32")
    cat = small_cat(seed=7)
    plan = tsb.Plan(**req)
    a = plan.assign(tsb.catalog_to_device(cat)).cpu().numpy()
    perm = np.random.default_rng(0).permutation(len(cat["pos"]))
    b = plan.assign(tsb.catalog_to_device({"pos": cat["pos"][perm]})).cpu().numpy()
    assert np.array_equal(a, b)


def test_assignment_crowded_cell():
    # 30k particles inside one cell on a tile corner plus a uniform background:
    # worst case for atomics on a single LDS address and for the bucket runs
    rng = np.random.default_rng(11)
    h = 1000.0 / 32
    crowd = (np.array([8.0, 15.0, 31.0]) + 0.9 * rng.random((30000, 3))) * h
    back = rng.random((5000, 3)) * 1000.0
    cat = {"pos": np.concatenate([crowd, back]).astype(np.float32)}
    _say("crowded cell")
    _assign_vs_oracle(box_request(n=32, precision="f64"), cat, 1e-12)


def test_assignment_edges_wrap():
    # positions on and just outside the box faces wrap periodically (box mode)
    rng = np.random.default_rng(12)
    L = 1000.0
    edge = np.array([0.0, L, -1e-3, L + 1e-3, np.nextafter(np.float32(L), np.float32(0)), 0.5 * L],
                    np.float32)
    pos = rng.choice(edge, size=(3000, 3)).astype(np.float32)
    pos = np.concatenate([pos, (rng.random((3000, 3)) * L).astype(np.float32)])
    _say("edges")
    _assign_vs_oracle(box_request(n=32, precision="f64"), {"pos": pos}, 1e-12)


def test_small_tiles_dense_fp32():
    # 16^3: 4^3 tiles, packed whole and as the parts of split tiles; 20k
    # particles make most tiles split
    req = box_request(n=16, precision="f32", n_bins=3, multipoles=[(0, 0, 0), (1, 1, 0), (2, 0, 2)])
    cat = small_cat(n=16, n_target=20000, seed=9)
    _say("small tiles dense", len(cat["pos"]))
    plan = tsb.Plan(**req)
    grids = plan.assign(tsb.catalog_to_device(cat)).cpu().numpy()
    op = oracle_plan(**req)
    _fp32_assignment_model(plan, op, cat, grids, est.assign_channels(op, cat)[0])
    plan, g, o = run_both(req, cat)
    mask = pair_mask(req["multipoles"], req["n_bins"])
    err = normwise_errors(g["B"], o["B"], mask)
    _say("small tiles errors", err)
    assert np.all(err <= 1e-4)
    # order-free fixed-point sums: a shuffled catalogue gives the same bits
    perm = np.random.default_rng(1).permutation(len(cat["pos"]))
    b = plan.measure(tsb.catalog_to_device({"pos": cat["pos"][perm]}))["B"]
    assert np.array_equal(np.nan_to_num(g["B"], nan=7.0), np.nan_to_num(b, nan=7.0))


@pytest.mark.parametrize("precision,tol", [("f32", 1e-4), ("f64", 1e-9)])
def test_radix3_grid(precision, tol):
    # 48^3 = 2^4 3: the transforms take the radix-4/2/3 passes
    req = box_request(n=48, n_bins=6, precision=precision)
    cat = small_cat(n=48, n_target=30000, seed=13)
    plan, g, o = run_both(req, cat)
    err = normwise_errors(g["B"], o["B"], pair_mask(req["multipoles"], req["n_bins"]))
    _say("48^3", precision, "errors", err, "M", plan.info.m)
    assert np.all(err <= tol)


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_box_mean_term_cancels_a_node_lattice(precision):
    # One unit-weight NGP particle on every node: with the box-mode node term
    # (reading R7) every channel is zero, so every multipole vanishes. The GPU
    # subtracts the term in spectrum space; the residue is set against B of a
    # uniform random catalogue of the same size on the same plan.
    n, box = 32, 1000.0
    req = box_request(n=n, box_len=box, assign_p=1, interlace=False, precision=precision,
                      multipoles=[(0, 0, 0), (1, 1, 0), (2, 0, 2), (1, 1, 2)], n_bins=6)
    j = np.arange(n, dtype=np.float64) * (box / n)
    X, Y, Z = np.meshgrid(j, j, j, indexing="ij")
    lattice = {"pos": np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float32), "w": None,
               "nbar": None}
    rng = np.random.default_rng(8)
    uniform = {"pos": (rng.random((n ** 3, 3)) * box).astype(np.float32), "w": None, "nbar": None}
    plan = tsb.Plan(**req)
    b_lat = plan.measure(tsb.catalog_to_device(lattice))["B"]
    b_uni = plan.measure(tsb.catalog_to_device(uniform))["B"]
    mask = pair_mask(req["multipoles"], req["n_bins"])
    for mu in range(len(req["multipoles"])):
        scale = np.max(np.abs(b_uni[mu][mask[mu]]))
        res = np.max(np.abs(b_lat[mu][mask[mu]]))
        _say("lattice", precision, req["multipoles"][mu], res, scale)
        assert res <= 1e-6 * scale


def test_one_pass_reduction_in_shell_groups():
    # {000, 110, 202} carries five slot kinds per shell: the one-pass reduction
    # transforms them one at a time, and with 14 shells on M = 64 it processes
    # each line's shells in two groups.
    n, box = 64, 1000.0
    kf = 2.0 * math.pi / box
    req = box_request(n=n, box_len=box, n_bins=14, dk=15.0 / 14.0 * kf,
                      multipoles=[(0, 0, 0), (1, 1, 0), (2, 0, 2)], precision="f32")
    cat = small_cat(n=n, box_len=box, n_target=60000, seed=12)
    plan, g, o = run_both(req, cat)
    assert plan.info.m == 64 and plan.info.n_fslots == 5
    mask = pair_mask(req["multipoles"], req["n_bins"])
    err = normwise_errors(g["B"], o["B"], mask)
    _say("grouped one-pass errors", err)
    assert np.all(err <= 1e-4)


def test_plan_k_eff_and_query_match_oracle():
    # k_eff (mean |k| of a shell, eq. 38) and N_mode of a plan on the device,
    # and the plan-based size query
    req = box_request(n=64, n_bins=8, dk=0.011, k_min=0.002)
    plan = tsb.Plan(**req)
    o = oracle_plan(**req)
    assert np.array_equal(np.array(plan.nmode), est.nmode(o))
    assert np.allclose(plan.k_eff, est.k_eff(o), rtol=1e-12, atol=0)
    ws, npairs, nm = plan.query()
    assert ws == plan.info.workspace_bytes and npairs == plan.info.n_outputs
    assert np.array_equal(np.array(nm), est.nmode(o))


def test_host_catalogue_equals_device_catalogue():
    # on_device = 0: the library copies the arrays; the result is bitwise the
    # device-catalogue result (survey mode: data and randoms, with w and nbar)
    req = box_request(n=32, n_bins=6, box_mode=False, P0=1e4, observer=(500.0, 500.0, 500.0),
                      multipoles=[(0, 0, 0), (2, 0, 2)])
    rng = np.random.default_rng(7)

    def shell(npts):
        v = rng.standard_normal((npts, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        return 500.0 + v * (200.0 + 200.0 * rng.random(npts))[:, None]

    data = {"pos": shell(5000), "w": 0.5 + rng.random(5000), "nbar": 1e-4 * (1 + rng.random(5000))}
    rand = {"pos": shell(20000), "w": None, "nbar": 1e-4 * (1 + rng.random(20000))}
    plan = tsb.Plan(**req)
    dev = plan.measure(tsb.catalog_to_device(data), tsb.catalog_to_device(rand))
    host = plan.measure(tsb.catalog_on_host(data), tsb.catalog_on_host(rand))
    mixed = plan.measure(tsb.catalog_on_host(data), tsb.catalog_to_device(rand))
    report("host catalogue vs device catalogue: alpha", host["alpha"], dev["alpha"])
    for r in (host, mixed):
        assert np.array_equal(np.nan_to_num(r["B"], nan=7.0), np.nan_to_num(dev["B"], nan=7.0))
        assert r["I"] == dev["I"] and r["alpha"] == dev["alpha"]
    o = est.measure(oracle_plan(**req), data, rand)
    err = normwise_errors(host["B"], o["B"], pair_mask(req["multipoles"], req["n_bins"]))
    report("host catalogue vs oracle", err)
    assert np.all(err <= 1e-4)


def test_survey_particle_outside_the_box_is_reported():
    # survey mode does not wrap positions: a galaxy past the box is an input
    # error (the kernels skip it; the measurement reports TSB_E_INPUT)
    req = box_request(n=32, n_bins=6, box_mode=False, observer=(500.0, 500.0, 500.0))
    rng = np.random.default_rng(9)
    data = {"pos": 300.0 + 400.0 * rng.random((3000, 3))}
    rand = {"pos": 300.0 + 400.0 * rng.random((9000, 3))}
    plan = tsb.Plan(**req)
    plan.measure(tsb.catalog_to_device(data), tsb.catalog_to_device(rand))   # inside: fine
    data["pos"][17] = (500.0, 1000.5, 500.0)
    with pytest.raises(tsb.TsbError) as e:
        plan.measure(tsb.catalog_to_device(data), tsb.catalog_to_device(rand))
    assert e.value.code == tsb.abi.TSB_E_INPUT and "outside" in str(e.value)


def test_particle_at_the_observer_is_reported():
    # a local LOS is undefined for a particle at the observer (eq. 34)
    req = box_request(n=32, n_bins=6)
    cat = small_cat(seed=12)
    pos = cat["pos"].copy()
    pos[5] = req["observer"]
    plan = tsb.Plan(**req)
    with pytest.raises(tsb.TsbError) as e:
        plan.measure(tsb.catalog_to_device({"pos": pos}))
    assert e.value.code == tsb.abi.TSB_E_INPUT and "observer" in str(e.value)
    # the plan measures normally afterwards
    g = plan.measure(tsb.catalog_to_device(cat))
    o = est.measure(oracle_plan(**req), cat)
    assert np.all(normwise_errors(g["B"], o["B"], pair_mask(req["multipoles"], req["n_bins"])) <= 1e-4)
