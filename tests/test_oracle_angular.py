"""Pins of the oracle's angular algebra against closed forms, symmetries,
library routines and the paper's printed tables (no GPU)."""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import angular as ang

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    return rows


def _three_j_000_closed(j1, j2, j3):
    """Closed form of (j1 j2 j3; 0 0 0) for J = j1+j2+j3 even (Edmonds 3.7.17)."""
    J = j1 + j2 + j3
    if J % 2 or j3 < abs(j1 - j2) or j3 > j1 + j2:
        return 0.0
    g = J // 2
    f = math.factorial
    return ((-1) ** g * math.sqrt(f(J - 2 * j1) * f(J - 2 * j2) * f(J - 2 * j3) / f(J + 1))
            * f(g) / (f(g - j1) * f(g - j2) * f(g - j3)))


@pytest.mark.parametrize("j1,j2,j3,val", [
    (0, 0, 0, 1.0), (1, 1, 0, -1.0 / math.sqrt(3.0)), (2, 0, 2, 1.0 / math.sqrt(5.0)),
    (2, 2, 0, 1.0 / math.sqrt(5.0)), (1, 1, 2, math.sqrt(2.0 / 15.0)), (4, 0, 4, 1.0 / 3.0)])
def test_h_of_table_multipoles(j1, j2, j3, val):
    assert ang.h_factor(j1, j2, j3) == pytest.approx(val, rel=1e-15, abs=1e-16)


def test_three_j_000_against_closed_form():
    for j1, j2, j3 in itertools.product(range(7), repeat=3):
        assert ang.wigner_3j(j1, j2, j3, 0, 0, 0) == pytest.approx(
            _three_j_000_closed(j1, j2, j3), rel=1e-14, abs=1e-15)


def test_three_j_jj0_closed_form():
    # (j j 0; m -m 0) = (-1)^(j-m)/sqrt(2j+1)
    for j in range(6):
        for m in range(-j, j + 1):
            assert ang.wigner_3j(j, j, 0, m, -m, 0) == pytest.approx(
                (-1) ** (j - m) / math.sqrt(2 * j + 1), rel=1e-14)


def test_three_j_symmetries():
    rng = np.random.default_rng(1)
    for _ in range(300):
        j1, j2 = rng.integers(0, 5, size=2)
        j3 = rng.integers(abs(j1 - j2), j1 + j2 + 1)
        m1 = rng.integers(-j1, j1 + 1)
        m2 = rng.integers(-j2, j2 + 1)
        m3 = -m1 - m2
        if abs(m3) > j3:
            continue
        w = ang.wigner_3j(j1, j2, j3, m1, m2, m3)
        sgn = (-1) ** (j1 + j2 + j3)
        # even (cyclic) permutation
        assert ang.wigner_3j(j2, j3, j1, m2, m3, m1) == pytest.approx(w, abs=1e-15)
        # odd permutation
        assert ang.wigner_3j(j2, j1, j3, m2, m1, m3) == pytest.approx(sgn * w, abs=1e-15)
        # sign flip of every m
        assert ang.wigner_3j(j1, j2, j3, -m1, -m2, -m3) == pytest.approx(sgn * w, abs=1e-15)


def test_three_j_orthogonality():
    for j1, j2 in [(1, 1), (2, 1), (2, 2), (3, 2), (4, 2)]:
        for j3 in range(abs(j1 - j2), j1 + j2 + 1):
            for j3p in range(abs(j1 - j2), j1 + j2 + 1):
                for m3 in range(-j3, j3 + 1):
                    m3p = m3
                    if abs(m3p) > j3p:
                        continue
                    s = sum((2 * j3 + 1) * ang.wigner_3j(j1, j2, j3, m1, m2, m3)
                            * ang.wigner_3j(j1, j2, j3p, m1, m2, m3p)
                            for m1 in range(-j1, j1 + 1) for m2 in range(-j2, j2 + 1))
                    assert s == pytest.approx(1.0 if j3 == j3p else 0.0, abs=1e-13)


def test_three_j_against_sympy():
    sympy_w = pytest.importorskip("sympy.physics.wigner")
    for j1, j2, j3 in itertools.product(range(5), repeat=3):
        for m1 in range(-j1, j1 + 1):
            for m2 in range(-j2, j2 + 1):
                m3 = -m1 - m2
                if abs(m3) > j3:
                    continue
                ref = float(sympy_w.wigner_3j(j1, j2, j3, m1, m2, m3))
                assert ang.wigner_3j(j1, j2, j3, m1, m2, m3) == pytest.approx(ref, abs=1e-14)


def _rand_units(n, seed):
    v = np.random.default_rng(seed).standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1)[:, None]


def test_y00_is_one():
    u = _rand_units(20, 2)
    assert np.allclose(ang.ylm(0, 0, u[:, 0], u[:, 1], u[:, 2]), 1.0, atol=0, rtol=1e-15)


def test_ylm_against_scipy():
    sp = pytest.importorskip("scipy.special")
    u = _rand_units(50, 3)
    theta = np.arccos(u[:, 2])
    phi = np.arctan2(u[:, 1], u[:, 0])
    for l in range(7):
        for m in range(-l, l + 1):
            if hasattr(sp, "sph_harm_y"):
                Y = sp.sph_harm_y(l, m, theta, phi)
            else:
                Y = sp.sph_harm(m, l, phi, theta)
            ref = math.sqrt(4.0 * math.pi / (2 * l + 1)) * Y
            got = ang.ylm(l, m, u[:, 0], u[:, 1], u[:, 2])
            assert np.allclose(got, ref, rtol=1e-12, atol=1e-13)


def test_addition_theorem():
    # App. A, eq. A2: L_l(x.y) = sum_m y_l^m(x) y_l^m*(y)
    a = _rand_units(40, 4)
    b = _rand_units(40, 5)
    mu = np.sum(a * b, axis=1)
    for l in range(8):
        s = sum(ang.ylm(l, m, *a.T) * np.conj(ang.ylm(l, m, *b.T)) for m in range(-l, l + 1))
        assert np.allclose(s, ang.legendre(l, mu), atol=1e-13)


def test_product_rule():
    # App. A, eq. A4: y_l1^m1 y_l2^m2 = sum_{l3 m3} (2 l3+1) 3j(l1 l2 l3;000) 3j(l1 l2 l3; m1 m2 m3) y_l3^m3*
    u = _rand_units(30, 6)
    for l1, l2 in [(1, 1), (2, 1), (2, 2), (3, 2), (4, 2)]:
        for m1 in range(-l1, l1 + 1):
            for m2 in range(-l2, l2 + 1):
                lhs = ang.ylm(l1, m1, *u.T) * ang.ylm(l2, m2, *u.T)
                rhs = np.zeros(len(u), complex)
                for l3 in range(abs(l1 - l2), l1 + l2 + 1):
                    m3 = -m1 - m2
                    if abs(m3) > l3:
                        continue
                    rhs += ((2 * l3 + 1) * ang.wigner_3j(l1, l2, l3, 0, 0, 0)
                            * ang.wigner_3j(l1, l2, l3, m1, m2, m3) * np.conj(ang.ylm(l3, m3, *u.T)))
                assert np.allclose(lhs, rhs, atol=1e-13)


def test_legendre_against_scipy():
    sp = pytest.importorskip("scipy.special")
    x = np.linspace(-1, 1, 41)
    for l in range(9):
        assert np.allclose(ang.legendre(l, x), sp.eval_legendre(l, x), atol=1e-14)


def test_table1_allowed_multipoles():
    rows = _load("table1_allowed_multipoles.txt")
    for L, l1, l2 in rows:
        assert ang.allowed_multipole(l1, l2, L)
    # for each L of Table 1, its first four entries are exactly the allowed pairs
    # with the smallest l1 + l2 (ties: l1 descending then listed order is immaterial)
    for L in (0, 2, 4):
        listed = {(l1, l2) for LL, l1, l2 in rows if LL == L}
        allowed = [(l1, l2) for l1 in range(8) for l2 in range(8) if ang.allowed_multipole(l1, l2, L)]
        s_max = max(a + b for a, b in listed)
        assert listed <= set(allowed)
        assert {p for p in allowed if sum(p) < s_max} <= listed
    for bad in [(1, 0, 0), (2, 0, 0), (2, 1, 2), (1, 1, 1), (0, 2, 2), (3, 0, 2)]:
        assert not ang.allowed_multipole(*bad)


def test_term_counts_printed_in_paper():
    for l1, l2, L, n_local, n_global in _load("term_counts.txt"):
        assert len(ang.reduction_terms(l1, l2, L, los="local")) == n_local
        assert len(ang.reduction_terms(l1, l2, L, los="global")) == n_global


def test_legendre_case_coefficients():
    # Sec. 3.1: N H 3j(l l 0; m -m 0) = (2l+1)(-1)^m, which turns the L=0
    # multipole into the Legendre coefficient (addition theorem)
    for l in range(6):
        for m in range(-l, l + 1):
            v = ang.n_factor(l, l, 0) * ang.h_factor(l, l, 0) * ang.wigner_3j(l, l, 0, m, -m, 0)
            assert v == pytest.approx((2 * l + 1) * (-1) ** m, rel=1e-14)
