"""The library's masked model (Sec. 6.2; host code behind the C ABI, no GPU)
against the FP64 oracle (oracle/masked.py): the 9j symbols over every
argument set the coupling of l <= 4 multipoles uses, the masked zeta of
eq. 63 with and without the integral constraint of eq. 64, and the Hankel
transform of eq. 68 over small and large k r (the spherical Bessel functions
in the series, downward and upward regimes). Tolerance 1e-12 relative."""
import itertools

import numpy as np
import pytest

import paper_1803_02132_amd as tsb
from oracle import angular as ang
from oracle import masked as mk

MULTS = [(0, 0, 0), (1, 1, 0), (2, 2, 0), (2, 0, 2), (0, 2, 2), (1, 1, 2), (2, 2, 2), (4, 0, 4), (3, 1, 2)]


def test_9j_matches_the_oracle_over_the_coupling_arguments():
    seen = 0
    for o, a, b in itertools.product(MULTS[:6], MULTS, MULTS):
        args = (*b, *a, *o)
        want = mk.wigner_9j(*args)
        got = tsb.wigner_9j(*args)
        assert abs(got - want) <= 1e-13 * max(1.0, abs(want))
        seen += want != 0.0
    assert seen > 50


def _fields(seed, n=11):
    rng = np.random.default_rng(seed)
    r = np.linspace(5.0, 105.0, n)
    w = np.full(n, r[1] - r[0])
    zeta = {m: rng.standard_normal((n, n)) for m in MULTS}
    Q = {m: 0.3 * rng.standard_normal((n, n)) for m in MULTS}
    Q[(0, 0, 0)] = 1.0 + 0.1 * rng.random((n, n))
    return r, w, zeta, Q


@pytest.mark.parametrize("integral", [False, True])
def test_masked_zeta_matches_the_oracle(integral):
    r, w, zeta, Q = _fields(5)
    model, window, out = MULTS, MULTS[:7], MULTS[:6]
    got, zb = tsb.masked_zeta(out, model, zeta, window, Q, r, w, integral_constraint=integral)
    want, zb_o = mk.masked_zeta(out, model, zeta, window, {m: Q[m] for m in window}, r, w, integral=integral)
    assert zb == pytest.approx(zb_o, rel=1e-12, abs=0.0 if integral else 1e-300)
    for m in out:
        scale = np.max(np.abs(want[m]))
        assert scale > 0
        assert np.max(np.abs(got[m] - want[m])) <= 1e-12 * scale


@pytest.mark.parametrize("l1,l2", [(0, 0), (1, 1), (2, 0), (0, 2), (2, 2), (4, 0), (3, 1), (4, 4)])
def test_masked_bispectrum_matches_the_oracle(l1, l2):
    rng = np.random.default_rng(l1 * 10 + l2)
    r = np.linspace(0.0, 180.0, 46)
    w = np.full(r.size, r[1] - r[0])
    zeta = rng.standard_normal((r.size, r.size))
    k = np.concatenate([[0.0, 1e-4, 0.003], np.linspace(0.01, 0.3, 15)])   # k r from 0 to 54
    got = tsb.masked_bispectrum(l1, l2, zeta, r, w, k)
    want = mk.masked_bispectrum(l1, l2, zeta, r, w, k)
    scale = np.max(np.abs(want))
    assert np.max(np.abs(got - want)) <= 1e-12 * scale


def test_masked_model_argument_errors():
    r, w, zeta, Q = _fields(6, n=4)
    with pytest.raises(tsb.TsbError) as e:   # the integral constraint needs Q_000
        tsb.masked_zeta([(0, 0, 0)], [(0, 0, 0)], zeta, [(1, 1, 0)], Q, r, w, integral_constraint=True)
    assert e.value.code == tsb.abi.TSB_E_ARG
    with pytest.raises(tsb.TsbError) as e:
        tsb.masked_bispectrum(1, 0, zeta[(0, 0, 0)], r, w, np.array([0.1]))
    assert e.value.code == tsb.abi.TSB_E_UNSUPPORTED
    with pytest.raises(tsb.TsbError) as e:
        tsb.wigner_9j(20, 0, 20, 0, 0, 0, 20, 0, 20)
    assert e.value.code == tsb.abi.TSB_E_UNSUPPORTED
    assert ang.h_factor(1, 1, 0) != 0.0
