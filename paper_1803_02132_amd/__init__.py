"""MI355X (gfx950) bispectrum multipoles B_{l1 l2 L}(k1, k2) with the FFT-based
TripoSH estimator of arXiv:1803.02132.

The computation lives in libtriposh.so (hand-written HIP kernels behind the C
ABI of include/triposh.h). This package holds the ctypes binding (``abi``) and
``Plan``, which only marshals arguments: torch provides device memory and the
stream.
"""
import numpy as np

from . import abi
from .abi import TsbError

__all__ = ["Plan", "Server", "TsbError", "abi", "catalog_on_host", "catalog_to_device", "measure_batch", "query"]

_PAIR = {"paper": abi.TSB_PAIRS_PAPER, "upper": abi.TSB_PAIRS_UPPER, "diagonal": abi.TSB_PAIRS_DIAGONAL,
         "all": abi.TSB_PAIRS_ALL}


_ESTIMATOR = {"bispectrum": abi.TSB_BISPECTRUM, "3pcf": abi.TSB_3PCF, "window": abi.TSB_WINDOW}
_VERTEX = {"x3": abi.TSB_VERTEX_X3, "x1": abi.TSB_VERTEX_X1, "x2": abi.TSB_VERTEX_X2}


def _axes(v, typ):
    return tuple(typ(x) for x in v) if hasattr(v, "__len__") else (typ(v),) * 3


def _request(n, box_len, multipoles, n_bins, dk=1.0, k_min=0.0, edges=None, origin=(0.0, 0.0, 0.0), assign_p=3,
             interlace=False, los="local", los_dir=(0.0, 0.0, 1.0), observer=(0.0, 0.0, 0.0), vertex="x3",
             box_mode=True, P0=0.0, precision="f32", pair_mode="paper", unfused=False, estimator="bispectrum",
             shot_noise=False, assign_tiles=False):
    """The C structs of a request. `n` and `box_len` are one value or three (per
    axis); `edges` (n_bins + 1 values) overrides k_min / dk. The returned tuple
    keeps the edges array alive."""
    grid = abi.tsb_grid((abi.ctypes.c_int32 * 3)(*_axes(n, int)), (abi.ctypes.c_double * 3)(*_axes(box_len, float)),
                        (abi.ctypes.c_double * 3)(*origin), int(assign_p), int(bool(interlace)))
    lo = abi.tsb_los(abi.TSB_LOS_LOCAL if los == "local" else abi.TSB_LOS_GLOBAL,
                     (abi.ctypes.c_double * 3)(*los_dir), (abi.ctypes.c_double * 3)(*observer), _VERTEX[vertex])
    earr = None
    if edges is not None:
        earr = (abi.ctypes.c_double * len(edges))(*[float(e) for e in edges])
    bins = abi.tsb_kbins(int(n_bins), float(k_min), float(dk), earr)
    mps = [abi.tsb_multipole(*map(int, m)) for m in multipoles]
    opts = abi.tsb_options(abi.TSB_FP64 if precision == "f64" else abi.TSB_FP32, _PAIR[pair_mode],
                           int(bool(box_mode)), float(P0), int(unfused), _ESTIMATOR[estimator],
                           int(bool(shot_noise)), int(assign_tiles))
    return grid, lo, bins, mps, opts, earr


def query(**kw):
    """Host-only validation and sizes of a request (no device needed):
    (info, N_mode per bin, k_eff per bin)."""
    grid, lo, bins, mps, opts, _keep = _request(**kw)
    info, nmode, keff = abi.tsb_request_query(grid, lo, bins, mps, opts, bins.n_bins)
    return info, np.array(nmode, dtype=np.int64), np.array(keff)


def catalog_to_device(cat, device="cuda"):
    """Host catalogue dict (pos (N,3) float32, optional w, nbar) -> dict of
    contiguous float32 torch tensors on the device (kept alive by the caller)."""
    import torch
    pos = np.ascontiguousarray(np.asarray(cat["pos"], np.float32).T)
    out = {k: torch.from_numpy(np.ascontiguousarray(pos[i])).to(device) for i, k in enumerate("xyz")}
    for k in ("w", "nbar"):
        v = cat.get(k)
        out[k] = None if v is None else torch.from_numpy(np.ascontiguousarray(np.asarray(v, np.float32))).to(device)
    return out


def catalog_on_host(cat):
    """Host catalogue dict (pos (N,3), optional w, nbar) -> dict of contiguous
    float32 numpy arrays; measured with on_device = 0 (the library copies them
    to the device)."""
    pos = np.ascontiguousarray(np.asarray(cat["pos"], np.float32).T)
    out = {k: np.ascontiguousarray(pos[i]) for i, k in enumerate("xyz")}
    for k in ("w", "nbar"):
        v = cat.get(k)
        out[k] = None if v is None else np.ascontiguousarray(np.asarray(v, np.float32))
    return out


def _cat_struct(dev):
    """tsb_catalog of a dict of device tensors (on_device = 1) or of host numpy
    arrays (on_device = 0)."""
    if dev is None:
        return None
    on_device = hasattr(dev["x"], "data_ptr")

    def ptr(t):
        if t is None:
            return None
        return t.data_ptr() if on_device else t.ctypes.data

    n = int(dev["x"].numel()) if on_device else int(dev["x"].size)
    return abi.tsb_catalog(ptr(dev["x"]), ptr(dev["y"]), ptr(dev["z"]), ptr(dev.get("w")), ptr(dev.get("nbar")),
                           n, int(on_device))


class Plan:
    """A measurement plan on the current device (see tsb_plan_create)."""

    def __init__(self, **kw):
        self.request = dict(kw)
        grid, lo, bins, mps, opts, _keep = _request(**kw)
        self.n_bins = bins.n_bins
        self.multipoles = [tuple(map(int, m)) for m in kw["multipoles"]]
        self.handle = abi.tsb_plan_create(grid, lo, bins, mps, opts)
        self.info = abi.tsb_plan_get_info(self.handle)
        self.nmode, self.k_eff = abi.tsb_plan_nmode(self.handle, self.n_bins)
        self.precision = kw.get("precision", "f32")

    def shot_noise(self):
        """The shot noise S that the last measure() subtracted (plans created with
        shot_noise=True) and its i = j != k term, each (n_mult, n_bins, n_bins)."""
        S = np.empty((len(self.multipoles), self.n_bins, self.n_bins), dtype=np.float64)
        Sij = np.empty_like(S)
        abi.tsb_plan_shot_noise(self.handle, S.ctypes.data, Sij.ctypes.data)
        return S, Sij

    def query(self):
        """tsb_plan_query: (workspace bytes, computed entries, N_mode per bin)."""
        return abi.tsb_plan_query(self.handle, self.n_bins)

    def channels(self):
        return [abi.tsb_plan_channel(self.handle, c) for c in range(self.info.n_channels)]

    def measure(self, data_dev, randoms_dev=None, stream=None):
        """Run the hot path on device catalogues (dicts of torch tensors).
        Returns dict(B=(n_mult, n_bins, n_bins) float64, I, alpha)."""
        import torch
        s = torch.cuda.current_stream() if stream is None else stream
        B = np.empty((len(self.multipoles), self.n_bins, self.n_bins), dtype=np.float64)
        I, alpha = abi.tsb_measure(self.handle, _cat_struct(data_dev), _cat_struct(randoms_dev),
                                   s.cuda_stream, B.ctypes.data)
        return {"B": B, "I": I, "alpha": alpha}

    def measure_noalloc(self, data_dev, randoms_dev=None, stream=None):
        """tsb_measure_noalloc: the same measurement with no device allocation
        (buffers in the library's static scratch). Device catalogues only."""
        import torch
        s = torch.cuda.current_stream() if stream is None else stream
        B = np.empty((len(self.multipoles), self.n_bins, self.n_bins), dtype=np.float64)
        I, alpha = abi.tsb_measure_noalloc(self.handle, _cat_struct(data_dev), _cat_struct(randoms_dev),
                                           s.cuda_stream, B.ctypes.data)
        return {"B": B, "I": I, "alpha": alpha}

    def assign(self, data_dev, randoms_dev=None, stream=None):
        """Assignment stage only: grids [copies][channel][Nx][Ny][Nz] as a torch tensor."""
        import torch
        s = torch.cuda.current_stream() if stream is None else stream
        copies = 1 + int(bool(self.request.get("interlace", False)))
        nx, ny, nz = _axes(self.request["n"], int)
        dt = torch.float64 if self.precision == "f64" else torch.float32
        out = torch.empty((copies, self.info.n_channels, nx, ny, nz), dtype=dt, device="cuda")
        abi.tsb_assign(self.handle, _cat_struct(data_dev), _cat_struct(randoms_dev), s.cuda_stream,
                       out.data_ptr())
        return out

    def autotune(self, data_dev, randoms_dev=None, stream=None, reps=3):
        """tsb_plan_autotune on these catalogues; returns the chosen schedule."""
        import torch
        s = torch.cuda.current_stream() if stream is None else stream
        return abi.tsb_plan_autotune(self.handle, _cat_struct(data_dev), _cat_struct(randoms_dev), s.cuda_stream,
                                     reps)

    def set_schedule(self, choice):
        """tsb_plan_set_schedule with a dict in the layout autotune() returns."""
        abi.tsb_plan_set_schedule(self.handle, choice)

    def set_graphs(self, enable):
        abi.tsb_plan_set_graphs(self.handle, enable)

    def close(self):
        if getattr(self, "handle", None) is not None:
            abi.tsb_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def measure_batch(plans, datas, randoms=None, stream=None):
    """tsb_measure_batch: item i measures datas[i] (randoms[i]) with plans[i].
    Returns a list of dict(B, I, alpha)."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    Bs = [np.empty((len(p.multipoles), p.n_bins, p.n_bins), dtype=np.float64) for p in plans]
    rs = None if randoms is None else [_cat_struct(r) for r in randoms]
    I, alpha = abi.tsb_measure_batch([p.handle for p in plans], [_cat_struct(d) for d in datas], rs,
                                     s.cuda_stream, [B.ctypes.data for B in Bs])
    return [{"B": B, "I": i, "alpha": a} for B, i, a in zip(Bs, I, alpha)]


class Server:
    """tsb_server_*: a request loop on the current device. Keeps each request's
    catalogue tensors and output array alive until the request is done."""

    def __init__(self, hbm_budget_bytes, max_slots):
        self.handle = abi.tsb_server_create(hbm_budget_bytes, max_slots)
        self._live = {}

    def submit(self, plan, data_dev, randoms_dev=None):
        B = np.empty((len(plan.multipoles), plan.n_bins, plan.n_bins), dtype=np.float64)
        t = abi.tsb_server_submit(self.handle, plan.handle, _cat_struct(data_dev), _cat_struct(randoms_dev),
                                  B.ctypes.data)
        self._live[t] = (B, data_dev, randoms_dev)
        return t

    def stats(self):
        """(most requests running at once, workspaces released)."""
        return abi.tsb_server_stats(self.handle)

    def poll(self, ticket):
        """(done, latency_s, B or None)."""
        done, lat = abi.tsb_server_poll(self.handle, ticket)
        return done, lat, (self._live.pop(ticket)[0] if done else None)

    def wait(self, ticket):
        """Block until done: (latency_s, B)."""
        lat = abi.tsb_server_wait(self.handle, ticket)
        return lat, self._live.pop(ticket)[0]

    def close(self):
        if getattr(self, "handle", None) is not None:
            abi.tsb_server_destroy(self.handle)
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wigner_9j(*l):
    """tsb_wigner_9j: {l0 l1 l2; l3 l4 l5; l6 l7 l8} (App. A)."""
    return abi.tsb_wigner_9j(*l)


def masked_zeta(out, model, zeta, window, Q, r=None, w=None, integral_constraint=True):
    """tsb_masked_zeta (Sec. 6.2, eqs. 63-64). zeta, Q: dicts multipole ->
    (n_r, n_r) arrays (r2 fastest). Returns ({out multipole: array}, zeta_bar)."""
    model, window, out = [tuple(map(int, m)) for m in model], [tuple(map(int, m)) for m in window], \
        [tuple(map(int, m)) for m in out]
    z = np.ascontiguousarray(np.stack([np.asarray(zeta[m], np.float64) for m in model]))
    q = np.ascontiguousarray(np.stack([np.asarray(Q[m], np.float64) for m in window]))
    n_r = z.shape[1]
    rr = None if r is None else np.ascontiguousarray(np.asarray(r, np.float64))
    ww = None if w is None else np.ascontiguousarray(np.asarray(w, np.float64))
    res = np.empty((len(out), n_r, n_r), np.float64)
    zbar = abi.tsb_masked_zeta(model, z.ctypes.data, window, q.ctypes.data,
                               None if rr is None else rr.ctypes.data, None if ww is None else ww.ctypes.data,
                               n_r, out, res.ctypes.data, integral_constraint)
    return {m: res[i] for i, m in enumerate(out)}, zbar


def masked_bispectrum(l1, l2, zeta, r, w, k):
    """tsb_masked_bispectrum (Sec. 6.2, eq. 68): B(k1, k2) on the k grid."""
    z = np.ascontiguousarray(np.asarray(zeta, np.float64))
    rr = np.ascontiguousarray(np.asarray(r, np.float64))
    ww = np.ascontiguousarray(np.asarray(w, np.float64))
    kk = np.ascontiguousarray(np.asarray(k, np.float64))
    B = np.empty((kk.size, kk.size), np.float64)
    abi.tsb_masked_bispectrum(l1, l2, z.ctypes.data, rr.ctypes.data, ww.ctypes.data, rr.size, kk.ctypes.data,
                              kk.size, B.ctypes.data)
    return B
