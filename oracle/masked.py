"""FP64 reference of the masked model of the three-point-function and
bispectrum multipoles (Sec. 6.2), plain and slow.

TEST INFRASTRUCTURE ONLY (see the package header).

What it computes (arXiv:1803.02132):

  wigner_9j            App. A, eq. A5: a sum over m4..m9 of five 3j symbols equals
                       (-1)^{l2+l5+l8} 3j(l1 l2 l3; m1 m2 m3) times the 9j symbol
                       {l1 l2 l3; l4 l5 l6; l7 l8 l9}; the sum is evaluated at the
                       first (m1, m2, m3) whose 3j does not vanish and divided by it.
  coupling             the bracket of eq. 63 times N_{l1 l2 L}: the weight of
                       Q_{l1'' l2'' L''} zeta_{l1' l2' L'} in the masked zeta_{l1 l2 L}.
  integral_constraint  eq. 64.
  masked_zeta          eq. 63.
  masked_bispectrum    eq. 68: (-i)^{l1+l2} (4 pi)^2 int dr1 r1^2 int dr2 r2^2
                       j_l1(k1 r1) j_l2(k2 r2) <zeta_{l1 l2 L}>(r1, r2).

Readings:
  M1  The r integrals of eqs. 64 and 68 are quadrature sums sum_i w_i f(r_i) on
      the caller's r grid with the caller's weights (measured zeta and Q live on
      r-bins).
  M2  The sums over (l1' l2' L') and (l1'' l2'' L'') of eq. 63 run over the
      model and window multipoles supplied; a multipole absent from a set is
      zero (the truncation the paper's App. F makes, keeping four of each).
  M3  Eq. 64 sums over the multipoles present in both sets.
  M4  A multipole with l1 < l2 is an ordinary entry of a set.

Pins (tests/test_oracle_masked.py): the 9j against sympy's routine and the
closed form of a 9j with a zero entry (a 6j); a uniform window (Q_000 only)
leaves every multipole at Q_000 zeta (eq. 65); the printed monopole expansion
Q_000 (zeta_000 - zeta_bar) + Q_110 zeta_110 / 3 + Q_220 zeta_220 / 5 (eq. 66);
the integral constraint's defining condition (eq. 61: the r1^2 r2^2 integral of
the masked monopole vanishes); the Hankel transform of Gaussians in closed form.
"""
import numpy as np
from scipy.special import spherical_jn

from . import angular as ang


def wigner_9j(l1, l2, l3, l4, l5, l6, l7, l8, l9):
    """{l1 l2 l3; l4 l5 l6; l7 l8 l9} from eq. A5 (integer arguments)."""
    w3 = ang.wigner_3j
    for m1 in range(-l1, l1 + 1):
        for m2 in range(-l2, l2 + 1):
            m3 = -m1 - m2
            if abs(m3) > l3:
                continue
            d = w3(l1, l2, l3, m1, m2, m3)
            if d != 0.0:
                break
        else:
            continue
        break
    else:
        return 0.0   # no (m1, m2, m3) with a non-zero 3j: the triad (l1 l2 l3) is not coupled
    total = 0.0
    for m4 in range(-l4, l4 + 1):
        for m5 in range(-l5, l5 + 1):
            m7 = m1 - m4                 # first 3j:  m4 - m1 + m7 = 0
            m6 = -m4 - m5                # second:   -m5 - m4 - m6 = 0
            m9 = m3 - m6                 # third:     m6 - m3 + m9 = 0
            m8 = -m7 - m9                # fourth:   -m7 - m9 - m8 = 0
            if m8 - m2 + m5 != 0:        # fifth:     m8 - m2 + m5 = 0
                continue
            if abs(m6) > l6 or abs(m7) > l7 or abs(m8) > l8 or abs(m9) > l9:
                continue
            sign = (-1) ** ((l4 - m4 + l5 - m5 + l6 - m6 + l7 - m7 + l8 - m8 + l9 - m9) % 2)
            total += sign * (w3(l4, l1, l7, m4, -m1, m7) * w3(l5, l4, l6, -m5, -m4, -m6)
                             * w3(l6, l3, l9, m6, -m3, m9) * w3(l7, l9, l8, -m7, -m9, -m8)
                             * w3(l8, l2, l5, m8, -m2, m5))
    return total / ((-1) ** ((l2 + l5 + l8) % 2) * d)


def coupling(out, model, window):
    """N_{l1l2L} {l1'' l2'' L''; l1' l2' L'; l1 l2 L}
    H_{l1l2L} H_{l1 l1' l1''} H_{l2 l2' l2''} H_{L L' L''} / (H_{l1'l2'L'} H_{l1''l2''L''})  (eq. 63)."""
    l1, l2, L = out
    a1, a2, aL = model
    b1, b2, bL = window
    h = ang.h_factor
    den = h(a1, a2, aL) * h(b1, b2, bL)
    if den == 0.0:
        return 0.0
    num = h(l1, l2, L) * h(l1, a1, b1) * h(l2, a2, b2) * h(L, aL, bL)
    if num == 0.0:
        return 0.0
    return ang.n_factor(l1, l2, L) * wigner_9j(b1, b2, bL, a1, a2, aL, l1, l2, L) * num / den


def _r2w(r, w):
    r = np.asarray(r, np.float64)
    return np.asarray(w, np.float64) * r * r


def integral_constraint(model, zeta, window, Q, r, w):
    """zeta_bar of eq. 64 (M1, M3). zeta, Q: dicts multipole -> (n_r, n_r) arrays."""
    q = _r2w(r, w)
    if (0, 0, 0) not in Q:
        raise ValueError("the integral constraint needs Q_000")
    den = q @ Q[(0, 0, 0)] @ q
    num = 0.0
    for mp in model:
        if mp in Q:
            l1, l2, L = mp
            num += (q @ (Q[mp] * zeta[mp]) @ q) / (ang.h_factor(l1, l2, L) ** 2 * ang.n_factor(l1, l2, L))
    return num / den


def masked_zeta(out, model, zeta, window, Q, r=None, w=None, integral=True):
    """<zeta_{out}>_model(r1, r2) of eq. 63, and zeta_bar (0 without the integral constraint)."""
    zbar = integral_constraint(model, zeta, window, Q, r, w) if integral else 0.0
    res = {}
    for o in out:
        acc = np.zeros_like(next(iter(zeta.values())))
        for a in model:
            for b in window:
                c = coupling(o, a, b)
                if c != 0.0:
                    acc = acc + c * Q[b] * zeta[a]
        if o in Q:
            acc = acc - Q[o] * zbar
        res[o] = acc
    return res, zbar


def masked_bispectrum(l1, l2, zeta, r, w, k):
    """eq. 68 on the r grid (M1): B(k1, k2), real for even l1 + l2."""
    q = _r2w(r, w)
    r = np.asarray(r, np.float64)
    k = np.asarray(k, np.float64)
    J1 = spherical_jn(l1, np.outer(k, r)) * q[None, :]
    J2 = spherical_jn(l2, np.outer(k, r)) * q[None, :]
    phase = (-1j) ** (l1 + l2)
    B = phase * (4.0 * np.pi) ** 2 * (J1 @ zeta @ J2.T)
    return B.real
