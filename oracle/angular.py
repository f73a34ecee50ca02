"""Angular algebra of the TripoSH decomposition, written out plainly in FP64.

TEST INFRASTRUCTURE ONLY (see the package header).

Contents and the passage each follows (arXiv:1803.02132):

* ``wigner_3j``       -- the Wigner 3j symbol that weights the m-sums of the
                         J=0 reduction (Sec. 2, eq. 11) and defines
                         H = 3j(l1 l2 L; 0 0 0). Evaluated with Racah's closed
                         formula in exact rational arithmetic, rounded once to
                         FP64 at the end.
* ``ylm``             -- the normalised harmonic y_l^m = sqrt(4 pi/(2l+1)) Y_l^m
                         (App. A, eq. A1) through its associated-Legendre form
                         (App. A, eq. A3). The associated Legendre function
                         carries the Condon-Shortley phase; any fixed phase
                         convention gives the same multipoles because every
                         term of eq. 11 carries (-1)^(m1+m2+M) = 1.
* ``legendre``        -- Legendre polynomials L_l (App. A, eq. A2).
* ``allowed_multipole`` -- the four conditions of Table 1 (Sec. 2).
* ``n_factor``, ``h_factor`` -- N_{l1 l2 L} = (2l1+1)(2l2+1)(2L+1) (Sec. 2, eq. 5)
                         and H_{l1 l2 L} (Sec. 2, after eq. 11).
* ``reduction_terms`` -- the (m1, m2, M) terms with non-zero 3j weight, for the
                         local-LOS estimator (Sec. 4.2, eq. 41) and the global
                         plane-parallel one (Sec. 4.4, eq. 52).

Pins (tests/test_oracle_angular.py): closed-form 3j values, the column
permutation / sign-flip symmetries and orthogonality of 3j, sympy's
``wigner_3j``; y_0^0 = 1, the addition theorem (eq. A2), the product rule
(eq. A4), scipy's spherical harmonics; Table 1 and the per-multipole term
counts printed in Sec. 4.4 (tests/golden/).
"""
from fractions import Fraction
from math import factorial, sqrt, pi

import numpy as np


def _racah_sum(j1, j2, j3, m1, m2, m3):
    """Exact rational sum over k of Racah's formula (integer arguments)."""
    total = Fraction(0)
    kmin = max(0, j2 - j3 - m1, j1 - j3 + m2)
    kmax = min(j1 + j2 - j3, j1 - m1, j2 + m2)
    for k in range(kmin, kmax + 1):
        den = (factorial(k) * factorial(j3 - j2 + k + m1) * factorial(j3 - j1 + k - m2)
               * factorial(j1 + j2 - j3 - k) * factorial(j1 - k - m1) * factorial(j2 - k + m2))
        total += Fraction((-1) ** k, den)
    return total


def wigner_3j_exact(j1, j2, j3, m1, m2, m3):
    """Return (sign, square) with 3j = sign * sqrt(square), square a Fraction.

    Racah's formula:
      (j1 j2 j3; m1 m2 m3) = (-1)^(j1-j2-m3) sqrt(Delta) sqrt(prod (j_i +- m_i)!) * S,
      Delta = (j1+j2-j3)!(j1-j2+j3)!(-j1+j2+j3)!/(j1+j2+j3+1)!,
    with S the alternating sum over k. Zero outside the selection rules
    (m1+m2+m3 = 0, triangle rule, |m_i| <= j_i).
    """
    js = (j1, j2, j3)
    ms = (m1, m2, m3)
    if any(int(j) != j or j < 0 for j in js) or any(int(m) != m for m in ms):
        raise ValueError("integer angular momenta only")
    if m1 + m2 + m3 != 0:
        return 0, Fraction(0)
    if any(abs(m) > j for j, m in zip(js, ms)):
        return 0, Fraction(0)
    if j3 < abs(j1 - j2) or j3 > j1 + j2:
        return 0, Fraction(0)
    delta = Fraction(factorial(j1 + j2 - j3) * factorial(j1 - j2 + j3) * factorial(-j1 + j2 + j3),
                     factorial(j1 + j2 + j3 + 1))
    facts = 1
    for j, m in zip(js, ms):
        facts *= factorial(j + m) * factorial(j - m)
    s = _racah_sum(j1, j2, j3, m1, m2, m3)
    if s == 0:
        return 0, Fraction(0)
    sign = (-1) ** ((j1 - j2 - m3) % 2) * (1 if s > 0 else -1)
    return sign, delta * facts * s * s


def wigner_3j(j1, j2, j3, m1, m2, m3):
    """Wigner 3j symbol in FP64 (exact rational square, one rounding, one sqrt)."""
    sign, sq = wigner_3j_exact(j1, j2, j3, m1, m2, m3)
    if sign == 0:
        return 0.0
    return sign * sqrt(float(sq))


def n_factor(l1, l2, L):
    """N_{l1 l2 L} = (2 l1 + 1)(2 l2 + 1)(2 L + 1) (Sec. 2, eq. 5)."""
    return (2 * l1 + 1) * (2 * l2 + 1) * (2 * L + 1)


def h_factor(l1, l2, L):
    """H_{l1 l2 L} = 3j(l1 l2 L; 0 0 0) (Sec. 2, after eq. 11)."""
    return wigner_3j(l1, l2, L, 0, 0, 0)


def allowed_multipole(l1, l2, L, require_ordered=True):
    """Table 1's four conditions: l1 >= l2; L even; |l1-l2| <= L <= l1+l2;
    l1 + l2 + L even. ``require_ordered=False`` drops the first one (the
    quantity with l1 < l2 is the transpose, B_{l1 l2 L}(k1,k2) = B_{l2 l1 L}(k2,k1))."""
    if min(l1, l2, L) < 0:
        return False
    if require_ordered and l1 < l2:
        return False
    if L % 2:
        return False
    if not (abs(l1 - l2) <= L <= l1 + l2):
        return False
    return (l1 + l2 + L) % 2 == 0


def _assoc_legendre(l, m, x):
    """Associated Legendre function P_l^m(x), m >= 0, Condon-Shortley phase,
    by the standard upward recurrence in l."""
    x = np.asarray(x, dtype=np.float64)
    somx2 = np.sqrt(np.maximum(0.0, (1.0 - x) * (1.0 + x)))
    pmm = np.ones_like(x)
    fact = 1.0
    for _ in range(m):
        pmm = -pmm * fact * somx2
        fact += 2.0
    if l == m:
        return pmm
    pmmp1 = x * (2 * m + 1) * pmm
    if l == m + 1:
        return pmmp1
    pll = pmmp1
    for ll in range(m + 2, l + 1):
        pll = ((2 * ll - 1) * x * pmmp1 - (ll + m - 1) * pmm) / (ll - m)
        pmm, pmmp1 = pmmp1, pll
    return pll


def ylm(l, m, ux, uy, uz):
    """Normalised spherical harmonic y_l^m at unit vectors (ux, uy, uz).

    App. A, eq. A3: y_l^m = (-1)^((m-|m|)/2) sqrt((l-|m|)!/(l+|m|)!) P_l^|m|(cos t) e^(i m phi).
    """
    ux = np.asarray(ux, dtype=np.float64)
    uy = np.asarray(uy, dtype=np.float64)
    uz = np.asarray(uz, dtype=np.float64)
    am = abs(m)
    if am > l:
        raise ValueError("|m| > l")
    cost = np.clip(uz, -1.0, 1.0)
    phi = np.arctan2(uy, ux)
    norm = sqrt(factorial(l - am) / factorial(l + am))
    sign = (-1) ** am if m < 0 else 1
    return sign * norm * _assoc_legendre(l, am, cost) * np.exp(1j * m * phi)


def legendre(l, x):
    """Legendre polynomial L_l(x) by Bonnet's recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if l == 0:
        return p0
    p1 = x.copy()
    for ll in range(1, l):
        p0, p1 = p1, ((2 * ll + 1) * x * p1 - ll * p0) / (ll + 1)
    return p1


def reduction_terms(l1, l2, L, los="local"):
    """Non-zero terms (m1, m2, M, 3j) of the m-sum.

    local LOS (Sec. 4.2, eq. 41): every (m1, m2, M) with m1 + m2 + M = 0.
    global LOS along z (Sec. 4.4, eq. 52): y_L^M*(z) = delta_M0, so M = 0, m2 = -m1.
    """
    out = []
    for m1 in range(-l1, l1 + 1):
        for m2 in range(-l2, l2 + 1):
            M = -m1 - m2
            if abs(M) > L:
                continue
            if los == "global" and M != 0:
                continue
            w = wigner_3j(l1, l2, L, m1, m2, M)
            if w != 0.0:
                out.append((m1, m2, M, w))
    return out
