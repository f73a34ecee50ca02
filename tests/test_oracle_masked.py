"""Pins of the oracle's masked model (no GPU): the 9j symbol of App. A against
sympy's routine and the 6j form of a 9j with a zero entry; a uniform window
leaves every multipole at Q_000 zeta (the leading term of eq. 65); the
printed monopole expansion (Sec. 6.2, eq. 66) with the coefficients 1/3 and
1/5; the defining condition of the integral constraint (eq. 61); the Hankel
transform of eq. 68 on Gaussians in closed form."""
import math
import random

import numpy as np
import pytest
from sympy.physics.wigner import wigner_6j, wigner_9j

from oracle import angular as ang
from oracle import masked as mk

MULTS = [(0, 0, 0), (1, 1, 0), (2, 2, 0), (2, 0, 2), (0, 2, 2), (1, 1, 2)]


def test_9j_against_sympy():
    rng = random.Random(3)
    for _ in range(80):
        c = [rng.randint(0, 4) for _ in range(9)]
        assert abs(mk.wigner_9j(*c) - float(wigner_9j(*c, prec=30))) <= 1e-13
    for c in [(2, 2, 2, 2, 2, 2, 2, 2, 2), (4, 2, 2, 2, 2, 0, 2, 0, 2), (1, 1, 2, 1, 1, 2, 2, 2, 0)]:
        assert abs(mk.wigner_9j(*c) - float(wigner_9j(*c, prec=30))) <= 1e-13


def test_9j_with_a_zero_is_a_6j():
    # {a b e; c d e; f f 0} = (-1)^{b+c+e+f} {a b e; d c f} / sqrt((2e+1)(2f+1))
    for (a, b, e, c, d, f) in [(1, 1, 0, 1, 1, 0), (2, 1, 1, 1, 2, 2), (2, 2, 2, 2, 2, 2), (3, 1, 2, 2, 2, 1),
                               (4, 2, 2, 2, 4, 2)]:
        want = (-1) ** (b + c + e + f) * float(wigner_6j(a, b, e, d, c, f)) / math.sqrt((2 * e + 1) * (2 * f + 1))
        assert abs(mk.wigner_9j(a, b, e, c, d, e, f, f, 0) - want) <= 1e-13


def _fields(seed, n=9):
    rng = np.random.default_rng(seed)
    r = np.linspace(10.0, 90.0, n)
    w = np.full(n, r[1] - r[0])
    zeta = {m: rng.standard_normal((n, n)) for m in MULTS}
    Q = {m: rng.standard_normal((n, n)) * 0.3 for m in MULTS}
    Q[(0, 0, 0)] = 1.0 + 0.1 * rng.random((n, n))
    return r, w, zeta, Q


def test_uniform_window_keeps_every_multipole():
    r, w, zeta, _ = _fields(1)
    q000 = np.full_like(zeta[(0, 0, 0)], 0.7)
    out, zbar = mk.masked_zeta(MULTS, MULTS, zeta, [(0, 0, 0)], {(0, 0, 0): q000}, integral=False)
    assert zbar == 0.0
    for m in MULTS:
        assert np.allclose(out[m], 0.7 * zeta[m], rtol=1e-13, atol=1e-14)


def test_printed_monopole_expansion():
    # Sec. 6.2, eq. 66: <zeta_000> = Q_000 (zeta_000 - zeta_bar) + Q_110 zeta_110 / 3 + Q_220 zeta_220 / 5
    # when the model and the window hold 000, 110 and 220
    sub = [(0, 0, 0), (1, 1, 0), (2, 2, 0)]
    r, w, zeta, Q = _fields(2)
    z = {m: zeta[m] for m in sub}
    q = {m: Q[m] for m in sub}
    out, zbar = mk.masked_zeta([(0, 0, 0)], sub, z, sub, q, r, w, integral=True)
    want = q[(0, 0, 0)] * (z[(0, 0, 0)] - zbar) + q[(1, 1, 0)] * z[(1, 1, 0)] / 3 + q[(2, 2, 0)] * z[(2, 2, 0)] / 5
    assert np.allclose(out[(0, 0, 0)], want, rtol=1e-12, atol=1e-13)


def test_integral_constraint_condition():
    # the integral constraint makes int dr1 r1^2 int dr2 r2^2 <zeta_000> vanish (Sec. 6.2, eq. 61)
    r, w, zeta, Q = _fields(3)
    out, zbar = mk.masked_zeta([(0, 0, 0)], MULTS, zeta, MULTS, Q, r, w, integral=True)
    q = w * r * r
    total = q @ out[(0, 0, 0)] @ q
    scale = q @ np.abs(Q[(0, 0, 0)] * zeta[(0, 0, 0)]) @ q
    assert abs(zbar) > 0
    assert abs(total) <= 1e-12 * scale


@pytest.mark.parametrize("l1,l2", [(0, 0), (2, 0), (1, 1), (2, 2)])
def test_hankel_of_gaussians(l1, l2):
    # int_0^inf r^{l+2} j_l(k r) exp(-r^2/2) dr = sqrt(pi/2) k^l exp(-k^2/2)
    r = np.linspace(0.0, 14.0, 4001)
    w = np.full(r.size, r[1] - r[0])
    w[0] = w[-1] = 0.5 * (r[1] - r[0])
    zeta = np.outer(r ** l1 * np.exp(-r * r / 2), r ** l2 * np.exp(-r * r / 2))
    k = np.array([0.1, 0.5, 1.0, 2.0, 3.0])
    B = mk.masked_bispectrum(l1, l2, zeta, r, w, k)
    g = lambda l: math.sqrt(math.pi / 2) * k ** l * np.exp(-k * k / 2)
    want = (-1) ** ((l1 + l2) // 2) * (4 * math.pi) ** 2 * np.outer(g(l1), g(l2))
    assert np.allclose(B, want, rtol=1e-9, atol=1e-12 * np.max(np.abs(want)))


def test_coupling_is_zero_off_the_triangles():
    # the 9j and the H symbols vanish unless every row and column couples
    assert mk.coupling((0, 0, 0), (2, 0, 2), (0, 0, 0)) == 0.0
    assert mk.coupling((2, 0, 2), (0, 0, 0), (0, 0, 0)) == 0.0
    assert abs(mk.coupling((2, 0, 2), (2, 0, 2), (0, 0, 0)) - 1.0) <= 1e-13
    assert abs(mk.coupling((0, 0, 0), (1, 1, 0), (1, 1, 0)) - 1.0 / 3.0) <= 1e-13
    assert ang.h_factor(1, 1, 0) ** 2 * ang.n_factor(1, 1, 0) == pytest.approx(3.0)
