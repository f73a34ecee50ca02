"""FP64 reference of the bispectrum-multipole estimator, plain and slow.

TEST INFRASTRUCTURE ONLY (see the package header).

What it computes (arXiv:1803.02132):

  O1  weights w = w_c / (1 + nbar P0)                      Sec. 5.2, eq. 54 (FKP factor)
  O2  alpha = sum_gal w / sum_ran w                        Sec. 4.1, after eq. 32
  O3  per-particle channel weights w_i y_L^M*(x_i^)         Sec. 4.1, eq. 34 (randoms x -alpha)
  O4  mass assignment (NGP/CIC/TSC) on a periodic grid      Sec. 4.2 (W_mass, eq. 39); App. C
  O5  forward DFT, e^{-ik.x}                                 Sec. 2 (Fourier convention)
  O6  divide by W_mass, interlace combine, Nyquist, DC      Sec. 4.2, eq. 39; readings R5, R6, R8
  O7  k-shells and N_mode                                   Sec. 4.2, eq. 38; Sec. 5.2
  O8  G_L^M(x) = int d3k/(2pi)^3 e^{ik.x} dn_L^M(k)/W        Sec. 4.2, eq. 42
  O9  F_l^m(x;k) = shell average of e^{ik.x} y_l^m*(k^) dn(k)/W   Sec. 4.2, eq. 42 with eq. 38
  O10 B = H sum_m 3j (N/I) int d3x F F G                    Sec. 4.2, eq. 41; Sec. 4.4, eq. 52
  O11 I = int d3x nbar^3 (survey) or (sum w)^3/V^2 (box)    Sec. 4.2, eq. 37; Sec. 4.4
  O12 the direct shell-averaged triangle sum of eq. 35     Sec. 4.2, eq. 35

The FFT route (O8-O10) and the direct triangle sum (O12) compute the same
number on a periodic grid: inserting sum_x e^{i(k1+k2+k3).x} = N^3 [k1+k2+k3 = 0
mod N] into eq. 41 gives eq. 35 with shells as in eq. 38. Tests check the two
against each other.

Discretisation. A grid of N^3 nodes at origin + j*H, H = L/N, periodic.
Assigned grid values D_j carry weight units (sum_j D_j = sum_i c_i), so
dn(k) = sum_j e^{-ik.x_j} D_j = numpy.fft.fftn(D). Then
  G(x)   = (N^3/V) ifftn(dn_L^M / W),
  F(x;b) = (N^3/N_mode(b)) ifftn(1_b y* dn/W),
  int d3x -> (V/N^3) sum_x,
so that all factors of V and N cancel in eq. 35.

Readings where the paper is silent or ambiguous:

  R1  Bins: [k_min + b dk, k_min + (b+1) dk), membership decided once per integer
      |n|^2 as floor((k_f sqrt(n^2) - k_min)/dk) in FP64; DC (n = 0) is in no shell.
  R2  Modes are indexed by signed n in (-N/2, N/2] per axis; N_mode counts the
      full grid.
  R3  Assignment kernels (Hockney & Eastwood) on nodes origin + j H, with grid
      coordinate u = (x - origin) * (N/L):
        NGP: j = floor(u + 1/2), weight 1;
        CIC: j = floor(u), d = u - j: (1-d) at j, d at j+1;
        TSC: j = floor(u + 1/2), d = u - j: (1/2)(1/2-d)^2 at j-1, 3/4 - d^2 at j,
             (1/2)(1/2+d)^2 at j+1.
      Node indices are taken mod N (periodic).
  R4  y_L^M*(x^) is applied per particle (eq. 34), x^ = (x - observer)/|x - observer|.
  R5  Interlacing (not in the paper): a second grid built from particles
      shifted by +H/2 along every axis (u2 = u + 1/2); the two transforms are
      combined as (D1 + e^{i pi (nx+ny+nz)/N} D2)/2 before dividing by W.
  R6  Modes with any index component equal to N/2 are set to zero in every field.
  R7  Periodic box (no randoms): dn = n - nbar with nbar = sum w / V. On the
      grid this subtracts (sum w / N^3) y_L^M*(x^_node) from every node of every
      channel (x^_node from the node position; the interlaced grid's node j sits
      at origin + (j - 1/2) H). The DC mode of the (0,0) channel is then set to 0.
  R8  Survey mode: I = v_c sum_j (alpha R_j / v_c)^3 with R the randoms assigned
      with weight w on the first grid (same scheme, not deconvolved).
      Box mode: I = (sum w)^3 / V^2 (Sec. 4.4 with weights).
  R9  FKP: w = w_c / (1 + nbar P0) when P0 > 0 and nbar is given, else w = w_c.
  R10 Global LOS along a unit vector d: only the (0,0) channel is gridded and
      G_L^M = y_L^M*(d) G_0^0 (Sec. 4.4 takes d = z, where y_L^M*(z) = delta_M0).
  R11 The multipole is the real part of eq. 41; its imaginary part vanishes for
      l1 + l2 + L even and is returned for checking.
  R12 LOS at the first or second vertex (App. B names x1, x2 and x3 as
      choices and gives no formula): the weight y_L^M*(x^) rides on the
      density of the first (x1) or second (x2) shell-filtered field instead of
      the third, so eq. 41 takes
        F_{l L}^{m M}(x; k) = shell average of e^{ik.x} y_l^m*(k^) dn_L^M(k)/W
      in place of F_l1^m1 (x1) or F_l2^m2 (x2), and G_0^0 in place of G_L^M;
      under a global LOS every vertex gives the same estimator.

The conventions R5 (interlace phase), R7 (box-mode node term) and R8 (value
of I) are definitions, each pinned by a property it implies: R5 by the exact
covariance of the interlaced field under a half-cell shift of the particles
along (1,1,1), R7 by the exact cancellation of every channel for particles on
the nodes, R8 by the closed form n-bar^3 V for a uniform density.
"""
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

from . import angular as ang


# ----------------------------------------------------------------------------
# Plan description


@dataclass
class Plan:
    """Everything eq. 41 needs besides the catalogue (Sec. 4.2, 5.2)."""
    n: int                       # grid points per side
    box_len: float               # L_box
    multipoles: Sequence[tuple]  # (l1, l2, L)
    n_bins: int
    dk: float
    k_min: float = 0.0
    origin: tuple = (0.0, 0.0, 0.0)
    assign_p: int = 3            # 1 NGP, 2 CIC, 3 TSC
    interlace: bool = False
    los: str = "local"           # "local" (vertex x3) or "global"
    los_dir: tuple = (0.0, 0.0, 1.0)
    observer: tuple = (0.0, 0.0, 0.0)
    box_mode: bool = True        # periodic box, no randoms
    P0: float = 0.0              # FKP; <= 0 disables
    edges: Optional[tuple] = None  # explicit bin edges (n_bins + 1); replaces k_min + b dk
    vertex: str = "x3"           # local LOS at the third vertex (main text), the first ("x1") or second ("x2", App. B)

    @property
    def volume(self):
        return self.box_len ** 3

    @property
    def k_f(self):
        return 2.0 * np.pi / self.box_len


# ----------------------------------------------------------------------------
# O1-O3: weights and channels


def fkp_weights(w_c, nbar, P0):
    """O1 (Sec. 5.2, eq. 54; R9): w = w_c * 1/(1 + nbar P0)."""
    w_c = np.asarray(w_c, dtype=np.float64)
    if nbar is None or P0 <= 0.0:
        return w_c.copy()
    return w_c / (1.0 + np.asarray(nbar, dtype=np.float64) * P0)


def alpha_ratio(w_gal, w_ran):
    """O2 (Sec. 4.1, after eq. 32): alpha = sum_gal w / sum_ran w."""
    return float(np.sum(np.asarray(w_gal, np.float64)) / np.sum(np.asarray(w_ran, np.float64)))


def channels(plan):
    """(L, M) of every y-weighted density field eq. 41 needs.

    Local LOS: every M in [-L, L] of every L in the multipole set (eq. 34),
    plus (0, 0), since every F field is built from dn = dn_0^0 (eq. 42).
    Global LOS: only (0, 0) (R10).
    """
    if plan.los == "global":
        return [(0, 0)]
    Ls = sorted({0} | {mp[2] for mp in plan.multipoles})
    return [(L, M) for L in Ls for M in range(-L, L + 1)]


def los_unit_vectors(pos, observer):
    """x^_i = (x_i - observer)/|x_i - observer| in FP64 (R4)."""
    d = np.asarray(pos, dtype=np.float64) - np.asarray(observer, dtype=np.float64)[None, :]
    r = np.sqrt(np.sum(d * d, axis=1))
    if np.any(r == 0.0):
        raise ValueError("a particle sits on the observer; its LOS is undefined")
    return d / r[:, None]


def channel_weights(pos, w, L, M, plan):
    """O3 (Sec. 4.1, eq. 34): c_i = w_i y_L^M*(x^_i) (complex)."""
    w = np.asarray(w, dtype=np.float64)
    if plan.los == "global":
        return w.astype(np.complex128)
    u = los_unit_vectors(pos, plan.observer)
    return w * np.conj(ang.ylm(L, M, u[:, 0], u[:, 1], u[:, 2]))


# ----------------------------------------------------------------------------
# O4: mass assignment


def grid_coordinate(pos, plan):
    """u = (x - origin) * (N / L) in FP64 (R3)."""
    inv_h = plan.n / plan.box_len
    return (np.asarray(pos, dtype=np.float64) - np.asarray(plan.origin, np.float64)[None, :]) * inv_h


def axis_stencil(u, p):
    """Per-axis node indices (unwrapped) and weights of the order-p kernel (R3).

    Returns (idx, wts) with shape (n_particles, p)."""
    if p == 1:
        j = np.floor(u + 0.5)
        return j[:, None].astype(np.int64), np.ones((u.size, 1))
    if p == 2:
        j = np.floor(u)
        d = u - j
        return (np.stack([j, j + 1], axis=1).astype(np.int64),
                np.stack([1.0 - d, d], axis=1))
    if p == 3:
        j = np.floor(u + 0.5)
        d = u - j
        return (np.stack([j - 1, j, j + 1], axis=1).astype(np.int64),
                np.stack([0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2], axis=1))
    raise ValueError("assign_p must be 1, 2 or 3")


def assign(pos, values, plan, shift=0.0):
    """O4: D_j = sum_i c_i W_p(x_j - x_i) on the periodic N^3 grid (complex128).

    ``shift`` is added to the grid coordinate (R5 uses +1/2)."""
    n = plan.n
    u = grid_coordinate(pos, plan) + shift
    values = np.asarray(values)
    stencils = [axis_stencil(u[:, a], plan.assign_p) for a in range(3)]
    re = np.zeros(n ** 3)
    im = np.zeros(n ** 3)
    p = plan.assign_p
    for a in range(p):
        for b in range(p):
            for c in range(p):
                ix = np.mod(stencils[0][0][:, a], n)
                iy = np.mod(stencils[1][0][:, b], n)
                iz = np.mod(stencils[2][0][:, c], n)
                wgt = stencils[0][1][:, a] * stencils[1][1][:, b] * stencils[2][1][:, c]
                flat = (ix * n + iy) * n + iz
                v = values * wgt
                re += np.bincount(flat, weights=np.real(v), minlength=n ** 3)
                if np.iscomplexobj(v):
                    im += np.bincount(flat, weights=np.imag(v), minlength=n ** 3)
    return (re + 1j * im).reshape(n, n, n)


def node_positions(plan, shift=0.0):
    """Physical positions of the grid nodes, shape (N, N, N, 3); ``shift`` in
    grid units is the offset of the particles (the node sits at -shift)."""
    n = plan.n
    h = plan.box_len / n
    j = (np.arange(n, dtype=np.float64) - shift) * h
    o = np.asarray(plan.origin, np.float64)
    X, Y, Z = np.meshgrid(j + o[0], j + o[1], j + o[2], indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def assign_channels(plan, data, randoms=None):
    """O1-O4 (and R7): the y-weighted density grids for every channel.

    ``data`` / ``randoms``: dict with 'pos' (n,3) and optional 'w', 'nbar'.
    Returns (grids, info) where grids[(L, M)] = [D_grid1, D_grid2 or None]."""
    pos = np.asarray(data["pos"], np.float64)
    w_c = data.get("w")
    w_c = np.ones(len(pos)) if w_c is None else np.asarray(w_c, np.float64)
    w = fkp_weights(w_c, data.get("nbar"), plan.P0)
    info = {"sum_w": float(np.sum(w))}
    if not plan.box_mode:
        rpos = np.asarray(randoms["pos"], np.float64)
        rw_c = randoms.get("w")
        rw_c = np.ones(len(rpos)) if rw_c is None else np.asarray(rw_c, np.float64)
        rw = fkp_weights(rw_c, randoms.get("nbar"), plan.P0)
        alpha = alpha_ratio(w, rw)
        info["alpha"] = alpha
        info["sum_w_ran"] = float(np.sum(rw))
    else:
        info["alpha"] = 0.0
    shifts = [0.0, 0.5] if plan.interlace else [0.0]
    grids = {}
    for (L, M) in channels(plan):
        per = []
        for s in shifts:
            D = assign(pos, channel_weights(pos, w, L, M, plan), plan, shift=s)
            if not plan.box_mode:
                D -= info["alpha"] * assign(rpos, channel_weights(rpos, rw, L, M, plan), plan, shift=s)
            else:
                # R7: subtract the mean density times y_L^M* at the node
                mean = info["sum_w"] / plan.n ** 3
                if plan.los == "global" or L == 0:
                    D -= mean
                else:
                    nodes = node_positions(plan, s).reshape(-1, 3)
                    u = los_unit_vectors(nodes, plan.observer)
                    D -= (mean * np.conj(ang.ylm(L, M, u[:, 0], u[:, 1], u[:, 2]))).reshape(D.shape)
            per.append(D)
        grids[(L, M)] = per
    if not plan.box_mode:
        R = assign(rpos, rw, plan, shift=0.0).real
        vc = plan.volume / plan.n ** 3
        info["I"] = float(np.sum((info["alpha"] * R) ** 3) / vc ** 2)   # R8, eq. 37
    else:
        info["I"] = info["sum_w"] ** 3 / plan.volume ** 2               # Sec. 4.4
    return grids, info


# ----------------------------------------------------------------------------
# O5-O7: spectra and shells


def signed_freq(n):
    """Signed integer frequencies of numpy's FFT ordering."""
    return np.fft.fftfreq(n, d=1.0 / n).round().astype(np.int64)


def mode_vectors(n):
    """Integer wave-vector grids (nx, ny, nz), each (N, N, N)."""
    f = signed_freq(n)
    return np.meshgrid(f, f, f, indexing="ij")


def mass_window(plan):
    """W_mass(k) = prod_i sinc(pi k_i / (2 k_N))^p = prod_i sinc(pi n_i / N)^p (eq. 39)."""
    nx, ny, nz = mode_vectors(plan.n)
    # numpy's sinc(x) = sin(pi x)/(pi x)
    return (np.sinc(nx / plan.n) * np.sinc(ny / plan.n) * np.sinc(nz / plan.n)) ** plan.assign_p


def spectra(plan, grids):
    """O5-O6: dn_L^M(k) = FFT(D)/W_mass, interlaced (R5), Nyquist zeroed (R6),
    DC of (0,0) zeroed in box mode (R7). Returns dict (L, M) -> (N,N,N) complex."""
    n = plan.n
    nx, ny, nz = mode_vectors(n)
    W = mass_window(plan)
    nyq = (np.abs(nx) == n // 2) | (np.abs(ny) == n // 2) | (np.abs(nz) == n // 2)
    out = {}
    for key, per in grids.items():
        D = np.fft.fftn(per[0])
        if plan.interlace:
            D2 = np.fft.fftn(per[1])
            D = 0.5 * (D + np.exp(1j * np.pi * (nx + ny + nz) / n) * D2)
        D = D / W
        D[nyq] = 0.0
        if plan.box_mode and key == (0, 0):
            D[0, 0, 0] = 0.0
        out[key] = D
    return out


def bin_of_n2(plan):
    """O7 (eq. 38, R1): bin index for every integer n^2 in [0, 3 (N/2)^2]; -1 if none.
    With explicit edges, bin b is [edges[b], edges[b+1])."""
    n2max = 3 * (plan.n // 2) ** 2
    n2 = np.arange(n2max + 1, dtype=np.float64)
    k = plan.k_f * np.sqrt(n2)
    if plan.edges is None:
        b = np.floor((k - plan.k_min) / plan.dk)
    else:
        e = np.asarray(plan.edges, dtype=np.float64)
        b = np.searchsorted(e, k, side="right") - 1.0   # the last edge not above k
    b = np.where((b >= 0) & (b < plan.n_bins), b, -1).astype(np.int64)
    b[0] = -1
    return b


def bin_grid(plan):
    """Bin index of every mode of the full grid (-1 outside every shell)."""
    nx, ny, nz = mode_vectors(plan.n)
    return bin_of_n2(plan)[nx * nx + ny * ny + nz * nz]


def nmode(plan):
    """N_mode(b): number of modes of the full grid in each shell (eq. 38)."""
    bg = bin_grid(plan)
    return np.array([int(np.sum(bg == b)) for b in range(plan.n_bins)], dtype=np.int64)


def k_eff(plan):
    """Mean |k| of the modes in each shell (for reporting)."""
    nx, ny, nz = mode_vectors(plan.n)
    k = plan.k_f * np.sqrt(nx * nx + ny * ny + nz * nz)
    bg = bin_grid(plan)
    return np.array([float(np.mean(k[bg == b])) if np.any(bg == b) else np.nan
                     for b in range(plan.n_bins)])


def mode_unit_vectors(plan):
    """n^ = n/|n| on the full grid (DC gets (0,0,1); it is in no shell)."""
    nx, ny, nz = mode_vectors(plan.n)
    r = np.sqrt(nx * nx + ny * ny + nz * nz).astype(np.float64)
    r[0, 0, 0] = 1.0
    ux, uy, uz = nx / r, ny / r, nz / r
    uz[0, 0, 0] = 1.0
    return ux, uy, uz


# ----------------------------------------------------------------------------
# O8-O11: FFT route


def g_field(plan, spec, L, M):
    """O8 (eq. 42): G_L^M(x) = (N^3/V) ifftn(dn_L^M/W); global LOS uses R10."""
    n = plan.n
    if plan.los == "global":
        d = np.asarray(plan.los_dir, np.float64)
        d = d / np.linalg.norm(d)
        yd = np.conj(ang.ylm(L, M, d[0], d[1], d[2]))
        return complex(yd) * (n ** 3 / plan.volume) * np.fft.ifftn(spec[(0, 0)])
    return (n ** 3 / plan.volume) * np.fft.ifftn(spec[(L, M)])


def f_field(plan, spec, l, m, b, bg=None, units=None, nm=None, src=(0, 0)):
    """O9 (eq. 42 with eq. 38): F_l^m(x; b) = (N^3/N_mode(b)) ifftn(1_b y_l^m*(k^) dn/W);
    with src = (L, M) the shell filter acts on dn_L^M (R12, LOS at x1 or x2)."""
    n = plan.n
    bg = bin_grid(plan) if bg is None else bg
    ux, uy, uz = mode_unit_vectors(plan) if units is None else units
    nm = nmode(plan) if nm is None else nm
    shell = (bg == b)
    A = np.zeros((n, n, n), dtype=np.complex128)
    A[shell] = np.conj(ang.ylm(l, m, ux[shell], uy[shell], uz[shell])) * spec[src][shell]
    return (n ** 3 / nm[b]) * np.fft.ifftn(A)


def reduce_fft(plan, spec, I, pairs=None):
    """O10 (eq. 41 / eq. 52): B[mu][b1][b2] and its imaginary part.

    ``pairs``: optional iterable of (b1, b2) to evaluate (others stay NaN).
    B = Re[(N H / I) sum_{m1 m2 M} 3j(l1 l2 L; m1 m2 M) (V/N^3) sum_x F F G].

    Pairs are evaluated row by row (one b1 at a time): the F fields of shell
    b1 and the products F(b1) G stay in memory while the row runs, the F
    fields of each b2 only while that pair runs, so a full-size grid needs a
    few dozen fields at a time. The terms of every pair are added in the
    order of ``angular.reduction_terms``. Under a global LOS a term whose
    weight y_L^M*(d) is exactly zero (every M != 0 for d = z) contributes
    exactly zero and is skipped."""
    n = plan.n
    nb = plan.n_bins
    bg = bin_grid(plan)
    units = mode_unit_vectors(plan)
    nm = nmode(plan)
    if pairs is None:
        pairs = [(b1, b2) for b1 in range(nb) for b2 in range(nb)]
    pairs = list(pairs)
    dv = plan.volume / n ** 3
    nmult = len(plan.multipoles)
    Bre = np.full((nmult, nb, nb), np.nan)
    Bim = np.full((nmult, nb, nb), np.nan)

    def los_weight(L, M):
        if plan.los != "global":
            return 1.0
        d = np.asarray(plan.los_dir, np.float64)
        d = d / np.linalg.norm(d)
        return complex(np.conj(ang.ylm(L, M, d[0], d[1], d[2])))

    # every (m1, m2, M) with m1+m2+M = 0 per multipole; under a global LOS the
    # weight y_L^M*(d) sits inside G_L^M (R10)
    mterms = []
    for (l1, l2, L) in plan.multipoles:
        terms = [t for t in ang.reduction_terms(l1, l2, L, los="local") if los_weight(L, t[2]) != 0]
        pref = ang.n_factor(l1, l2, L) * ang.h_factor(l1, l2, L) / I
        mterms.append((l1, l2, L, terms, pref))
    gcache = {}

    def G(L, M):
        if (L, M) not in gcache:
            gcache[(L, M)] = g_field(plan, spec, L, M)
        return gcache[(L, M)]

    def shell_fields(b, cache):
        def F(l, m, src=(0, 0)):
            if (l, m, src) not in cache:
                cache[(l, m, src)] = f_field(plan, spec, l, m, b, bg, units, nm, src)
            return cache[(l, m, src)]
        return F

    first_vertex = plan.vertex == "x1" and plan.los != "global"   # R12
    second_vertex = plan.vertex == "x2" and plan.los != "global"

    for b1 in sorted({p[0] for p in pairs}):
        f1 = {}
        F1 = shell_fields(b1, f1)
        prod = {}   # (mu, term index) -> F_l1^m1(x; b1) G_L^M(x)
        for b2 in sorted({p[1] for p in pairs if p[0] == b1}):
            F2 = F1 if b2 == b1 else shell_fields(b2, {})
            for mu, (l1, l2, L, terms, pref) in enumerate(mterms):
                acc = 0j
                for t, (m1, m2, M, w3j) in enumerate(terms):
                    if (mu, t) not in prod:
                        if first_vertex:
                            prod[(mu, t)] = (F1(l1, m1, (L, M)) * G(0, 0)).ravel()
                        elif second_vertex:
                            prod[(mu, t)] = (F1(l1, m1) * G(0, 0)).ravel()
                        else:
                            prod[(mu, t)] = (F1(l1, m1) * G(L, M)).ravel()
                    f2 = F2(l2, m2, (L, M)) if second_vertex else F2(l2, m2)
                    acc += w3j * dv * np.dot(prod[(mu, t)], f2.ravel())
                Bre[mu, b1, b2] = (pref * acc).real
                Bim[mu, b1, b2] = (pref * acc).imag
        del f1, prod
    return Bre, Bim


def measure(plan, data, randoms=None, pairs=None):
    """O1-O11 end to end. Returns dict with B (real), B_imag, I, alpha, nmode, k_eff."""
    grids, info = assign_channels(plan, data, randoms)
    spec = spectra(plan, grids)
    Bre, Bim = reduce_fft(plan, spec, info["I"], pairs=pairs)
    return {"B": Bre, "B_imag": Bim, "I": info["I"], "alpha": info["alpha"],
            "sum_w": info["sum_w"], "nmode": nmode(plan), "k_eff": k_eff(plan),
            "spectra": spec, "grids": grids}


# ----------------------------------------------------------------------------
# O12: direct triangle sum


def brute_force(plan, spec, I, pairs=None, chunk=4096):
    """O12 (eq. 35 with eq. 38): for each multipole and shell pair,
    (N H/I) sum_m 3j (1/(N_mode1 N_mode2)) sum_{n1 in b1} sum_{n2 in b2}
        y_l1^m1*(n1^) y_l2^m2*(n2^) dn(n1) dn(n2) dn_L^M(n3),  n3 = -n1-n2 mod N.
    Global LOS: dn_L^M = y_L^M*(d) dn (R10). LOS at x1 (R12): dn_L^M(n1)
    dn(n2) dn(n3) in place of dn(n1) dn(n2) dn_L^M(n3); at x2: dn(n1)
    dn_L^M(n2) dn(n3)."""
    n = plan.n
    nb = plan.n_bins
    bg = bin_grid(plan)
    nx, ny, nz = mode_vectors(n)
    ux, uy, uz = mode_unit_vectors(plan)
    if pairs is None:
        pairs = [(b1, b2) for b1 in range(nb) for b2 in range(nb)]
    shells = {}
    for b in range(nb):
        sel = np.nonzero(bg == b)
        shells[b] = (np.stack([nx[sel], ny[sel], nz[sel]], axis=1),
                     ux[sel], uy[sel], uz[sel], spec[(0, 0)][sel])
    nmult = len(plan.multipoles)
    Bre = np.full((nmult, nb, nb), np.nan)
    Bim = np.full((nmult, nb, nb), np.nan)
    for mu, (l1, l2, L) in enumerate(plan.multipoles):
        terms = ang.reduction_terms(l1, l2, L, los="local")
        pref = ang.n_factor(l1, l2, L) * ang.h_factor(l1, l2, L) / I
        for (b1, b2) in pairs:
            v1, x1, y1, z1, d1 = shells[b1]
            v2, x2, y2, z2, d2 = shells[b2]
            if len(d1) == 0 or len(d2) == 0:
                continue
            tot = 0j
            for (m1, m2, M, w3j) in terms:
                if plan.los == "global":
                    d = np.asarray(plan.los_dir, np.float64)
                    d = d / np.linalg.norm(d)
                    c3 = complex(np.conj(ang.ylm(L, M, d[0], d[1], d[2])))
                    if c3 == 0:
                        continue
                    s3 = spec[(0, 0)]
                else:
                    c3 = 1.0
                    s3 = spec[(L, M)]
                d1, d2 = shells[b1][4], shells[b2][4]
                if plan.vertex in ("x1", "x2") and plan.los != "global":
                    s3 = spec[(0, 0)]
                    if plan.vertex == "x1":
                        d1 = spec[(L, M)][np.nonzero(bg == b1)]
                    else:
                        d2 = spec[(L, M)][np.nonzero(bg == b2)]
                a1 = np.conj(ang.ylm(l1, m1, x1, y1, z1)) * d1
                a2 = np.conj(ang.ylm(l2, m2, x2, y2, z2)) * d2
                s = 0j
                for i0 in range(0, len(a1), chunk):
                    n1 = v1[i0:i0 + chunk]
                    n3 = np.mod(-(n1[:, None, :] + v2[None, :, :]), n)
                    c = s3[n3[..., 0], n3[..., 1], n3[..., 2]]
                    s += np.sum(a1[i0:i0 + chunk, None] * a2[None, :] * c)
                tot += w3j * c3 * s
            val = pref * tot / (len(d1) * len(d2))
            Bre[mu, b1, b2] = val.real
            Bim[mu, b1, b2] = val.imag
    return Bre, Bim
