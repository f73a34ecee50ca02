"""Seeded lognormal mocks (input generation only).

Recipe (the stand-in for the paper's galaxy catalogues and mocks, which are not
available here; every random number comes from numpy's PCG64 with the seed):

1. Gaussian field on an n^3 grid of side L: white noise eps ~ N(0,1) per cell,
   G_hat = rfftn(eps) sqrt(P(k)/v_c), G_hat(0) = 0, G = irfftn(G_hat), with
   P(k) = 2e4 (k/0.05)^-1.5 (Mpc/h)^3.
2. Lognormal contrast d = exp(G - s^2/2) - 1, s^2 the sample variance of G.
3. Poisson counts with mean nbar v_c (1 + d), positions uniform inside the cell.
4. Optional linear Kaiser displacement: psi(k) = i k G_hat/(b k^2), read at the
   particle's cell, x_s = x + f (psi . e) e with e the unit vector from the
   observer (local LOS) or a fixed direction (plane-parallel); periodic wrap.
5. Survey variant: a box centred on the observer, galaxies kept where
   r_min <= r <= r_max and z >= z_obs (half sky), uniform randoms in the same
   mask, nbar(r) from a radial histogram of the randoms scaled by N_d/N_r.
"""
import numpy as np


def power_law_pk(k, amp=2.0e4, k0=0.05, slope=-1.5):
    """P(k) = amp (k/k0)^slope; zero at k = 0."""
    k = np.asarray(k, dtype=np.float64)
    out = np.zeros_like(k)
    nz = k > 0
    out[nz] = amp * (k[nz] / k0) ** slope
    return out


def _kgrid(n, box_len):
    kf = 2.0 * np.pi / box_len
    kx = np.fft.fftfreq(n, d=1.0 / n) * kf
    kz = np.fft.rfftfreq(n, d=1.0 / n) * kf
    return np.meshgrid(kx, kx, kz, indexing="ij")


def gaussian_field(n, box_len, rng, pk=power_law_pk):
    """Step 1: real Gaussian field and its rfft (float64)."""
    vc = (box_len / n) ** 3
    eps = rng.standard_normal((n, n, n))
    KX, KY, KZ = _kgrid(n, box_len)
    k = np.sqrt(KX * KX + KY * KY + KZ * KZ)
    ghat = np.fft.rfftn(eps) * np.sqrt(pk(k) / vc)
    ghat[0, 0, 0] = 0.0
    g = np.fft.irfftn(ghat, s=(n, n, n), axes=(0, 1, 2))
    return g, ghat


def _to_f32_in_box(pos, box_len):
    """Wrap into [0, L) and convert to float32 without rounding up to L."""
    pos = np.mod(pos, box_len)
    p32 = pos.astype(np.float32)
    L32 = np.float32(box_len)
    p32 = np.where(p32 >= L32, p32 - L32, p32)
    return p32


def lognormal_box(n, box_len, n_target, seed, rsd=None, f=0.75, bias=2.0,
                  observer=None, los_dir=(0.0, 0.0, 1.0), pk=power_law_pk):
    """Steps 1-4 in a periodic box.

    rsd: None (real space), "local" (LOS from ``observer``) or "global" (along
    ``los_dir``). Returns dict(pos=(N_p,3) float32, w=None, nbar=None)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g, ghat = gaussian_field(n, box_len, rng, pk)
    var = g.var()
    delta = np.exp(g - 0.5 * var) - 1.0
    h = box_len / n
    nbar = n_target / box_len ** 3
    lam = nbar * h ** 3 * (1.0 + delta)
    counts = rng.poisson(lam.ravel())
    cells = np.repeat(np.arange(n ** 3, dtype=np.int64), counts)
    ix, iy, iz = np.unravel_index(cells, (n, n, n))
    base = np.stack([ix, iy, iz], axis=1).astype(np.float64) * h
    pos = base + rng.random((cells.size, 3)) * h
    if rsd is not None:
        KX, KY, KZ = _kgrid(n, box_len)
        k2 = KX * KX + KY * KY + KZ * KZ
        k2[0, 0, 0] = 1.0
        psi = np.empty((cells.size, 3))
        for a, K in enumerate((KX, KY, KZ)):
            comp = np.fft.irfftn(1j * K * ghat / (bias * k2), s=(n, n, n), axes=(0, 1, 2))
            psi[:, a] = comp.ravel()[cells]
        if rsd == "local":
            e = pos - np.asarray(observer, np.float64)[None, :]
            e /= np.sqrt(np.sum(e * e, axis=1))[:, None]
        elif rsd == "global":
            d = np.asarray(los_dir, np.float64)
            e = np.broadcast_to(d / np.linalg.norm(d), pos.shape)
        else:
            raise ValueError("rsd must be None, 'local' or 'global'")
        pos = pos + f * np.sum(psi * e, axis=1)[:, None] * e
    return {"pos": _to_f32_in_box(pos, box_len), "w": None, "nbar": None}


def _uniform_in_mask(n_pts, r_min, r_max, centre, rng):
    """Uniform points in the half shell r_min <= r <= r_max, z >= centre_z."""
    u = rng.random(n_pts)
    r = np.cbrt(r_min ** 3 + u * (r_max ** 3 - r_min ** 3))
    cost = rng.random(n_pts)                     # upper hemisphere
    phi = 2.0 * np.pi * rng.random(n_pts)
    sint = np.sqrt(1.0 - cost * cost)
    d = np.stack([sint * np.cos(phi), sint * np.sin(phi), cost], axis=1)
    return np.asarray(centre, np.float64)[None, :] + r[:, None] * d


def survey_catalogue(n, box_len, n_data, seed, r_min, r_max, random_factor=10,
                     nbar_bins=50, f=0.75, bias=2.0, pk=power_law_pk):
    """Step 5: masked data (Kaiser about the box centre) plus uniform randoms.

    Returns (data, randoms) dicts with pos (float32), w = None and nbar (float32)."""
    centre = np.full(3, 0.5 * box_len)
    v_mask = 0.5 * 4.0 / 3.0 * np.pi * (r_max ** 3 - r_min ** 3)
    n_box = n_data * box_len ** 3 / v_mask
    cat = lognormal_box(n, box_len, n_box, seed, rsd="local", f=f, bias=bias,
                        observer=centre, pk=pk)
    pos = cat["pos"].astype(np.float64)
    d = pos - centre[None, :]
    r = np.sqrt(np.sum(d * d, axis=1))
    keep = (r >= r_min) & (r <= r_max) & (d[:, 2] >= 0.0)
    dpos = pos[keep]
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    rpos = _uniform_in_mask(random_factor * len(dpos), r_min, r_max, centre, rng)
    # nbar(r) from the randoms: radial histogram scaled to the data count
    edges = np.linspace(r_min, r_max, nbar_bins + 1)
    hist, _ = np.histogram(np.sqrt(np.sum((rpos - centre) ** 2, axis=1)), bins=edges)
    shell_v = 0.5 * 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    nbar_r = hist * (len(dpos) / len(rpos)) / shell_v

    def nbar_at(p):
        rr = np.sqrt(np.sum((p - centre) ** 2, axis=1))
        idx = np.clip(np.searchsorted(edges, rr, side="right") - 1, 0, nbar_bins - 1)
        return nbar_r[idx].astype(np.float32)

    data = {"pos": _to_f32_in_box(dpos, box_len), "w": None, "nbar": nbar_at(dpos)}
    rand = {"pos": _to_f32_in_box(rpos, box_len), "w": None, "nbar": nbar_at(rpos)}
    return data, rand


def to_soa(cat):
    """(N,3) float32 positions -> contiguous x, y, z float32 arrays."""
    p = np.ascontiguousarray(np.asarray(cat["pos"], np.float32).T)
    return p[0], p[1], p[2]


# ----------------------------------------------------------------------------
# Named workloads (grid, box, particles, LOS, bins, multipoles)

WORKLOADS = {
    # 32^3 box, L = 1000, 20k particles, CIC, plane-parallel LOS along z,
    # {000, 202}, 8 bins of width 2 k_f from 0, FP64
    "box32": dict(n=32, box_len=1000.0, n_target=20000, assign_p=2, interlace=False,
                  los="global", multipoles=[(0, 0, 0), (2, 0, 2)], n_bins=8,
                  dk=2.0 * 2.0 * np.pi / 1000.0, k_min=0.0, rsd="global", precision="f64"),
    # 128^3 box, L = 1000, 500k particles, Kaiser along a local LOS from an
    # observer 1500 Mpc/h below the box centre, TSC + interlacing,
    # {000, 110, 202, 112}, 20 bins of dk = 0.01
    "box128": dict(n=128, box_len=1000.0, n_target=500000, assign_p=3, interlace=True,
                   los="local", observer=(500.0, 500.0, -1000.0),
                   multipoles=[(0, 0, 0), (1, 1, 0), (2, 0, 2), (1, 1, 2)], n_bins=20,
                   dk=0.01, k_min=0.0, rsd="local", precision="f32"),
    # the same recipe on a 256^3 grid with {000, 202}: one mock of the throughput
    # workload (particle count log-uniform in [3e5, 3e6] from the seed)
    "box256": dict(n=256, box_len=1000.0, n_target=None, assign_p=3, interlace=True,
                   los="local", observer=(500.0, 500.0, -1000.0),
                   multipoles=[(0, 0, 0), (2, 0, 2)], n_bins=20, dk=0.01, k_min=0.0,
                   rsd="local", precision="f32"),
    # survey window: 256^3 grid, L = 2000, 2M galaxies in the half shell
    # 500 <= r <= 1000 about the box centre (the observer), 10x randoms, FKP
    # weights with P0 = 1e4, {000, 202, 112, 404}, 25 bins of dk = 0.008
    # (up to about half the Nyquist frequency), TSC + interlacing
    "survey256": dict(n=256, box_len=2000.0, n_data=2_000_000, r_min=500.0, r_max=1000.0,
                      random_factor=10, P0=1.0e4, assign_p=3, interlace=True, los="local",
                      observer=(1000.0, 1000.0, 1000.0),
                      multipoles=[(0, 0, 0), (2, 0, 2), (1, 1, 2), (4, 0, 4)], n_bins=25,
                      dk=0.008, k_min=0.0, precision="f32"),
}


def headline_particle_count(seed):
    """N_p = floor(3e5 * 10^U), U ~ U(0,1) drawn from the seed."""
    rng = np.random.Generator(np.random.PCG64(10_000 + seed))
    return int(np.floor(3.0e5 * 10.0 ** rng.random()))


def survey_workload(name, seed=0, n_data=None):
    """Build (spec, data, randoms) for a named survey workload (step 5)."""
    spec = dict(WORKLOADS[name])
    if n_data is not None:
        spec["n_data"] = n_data
    data, rand = survey_catalogue(spec["n"], spec["box_len"], spec["n_data"], seed, spec["r_min"],
                                  spec["r_max"], random_factor=spec["random_factor"])
    return spec, data, rand


def workload(name, seed=0, n_target=None, n=None):
    """Build (spec, catalogue) for a named workload. ``n_target`` / ``n`` override
    the particle count / grid (for small test variants)."""
    spec = dict(WORKLOADS[name])
    if n is not None:
        spec["n"] = n
    if n_target is None:
        n_target = spec["n_target"] if spec["n_target"] is not None else headline_particle_count(seed)
    spec["n_target"] = n_target
    cat = lognormal_box(spec["n"], spec["box_len"], n_target, seed, rsd=spec["rsd"],
                        observer=spec.get("observer"))
    return spec, cat
