"""ctypes binding of include/triposh.h: the C entry points under the same names,
argument marshalling only. Every computation runs in libtriposh.so; if the
library is missing this module raises on import."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtriposh.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "(or python -m paper_1803_02132_amd.build)")
# One HIP runtime per process. torch ships its own libamdhip64 whose file name
# (libamdhip64.so) differs from the soname the library asks for
# (libamdhip64.so.7): with torch loaded first the library binds to torch's
# runtime; loaded first itself, it would pull in a second runtime that does not
# see the device torch initialises. So torch is imported before the library.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

TSB_OK, TSB_E_ARG, TSB_E_UNSUPPORTED, TSB_E_NOMEM, TSB_E_INPUT, TSB_E_DEVICE = 0, -1, -2, -3, -4, -5
TSB_E_BUSY, TSB_E_CANCELLED = -6, -7
TSB_LOS_GLOBAL, TSB_LOS_LOCAL = 0, 1
TSB_NGP, TSB_CIC, TSB_TSC = 1, 2, 3
TSB_FP32, TSB_FP64 = 0, 1
TSB_PAIRS_PAPER, TSB_PAIRS_UPPER, TSB_PAIRS_DIAGONAL, TSB_PAIRS_ALL = 0, 1, 2, 3
TSB_VERTEX_X3, TSB_VERTEX_X1, TSB_VERTEX_X2 = 0, 1, 2
TSB_BISPECTRUM, TSB_3PCF, TSB_WINDOW = 0, 1, 2

_STATUS = {TSB_E_ARG: "TSB_E_ARG", TSB_E_UNSUPPORTED: "TSB_E_UNSUPPORTED", TSB_E_NOMEM: "TSB_E_NOMEM",
           TSB_E_INPUT: "TSB_E_INPUT", TSB_E_DEVICE: "TSB_E_DEVICE", TSB_E_BUSY: "TSB_E_BUSY",
           TSB_E_CANCELLED: "TSB_E_CANCELLED"}


class TsbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class tsb_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("box_len", ctypes.c_double * 3), ("origin", ctypes.c_double * 3),
                ("assign_p", ctypes.c_int32), ("interlace", ctypes.c_int32)]


class tsb_los(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dir", ctypes.c_double * 3), ("observer", ctypes.c_double * 3),
                ("vertex", ctypes.c_int32)]


class tsb_kbins(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("k_min", ctypes.c_double), ("dk", ctypes.c_double),
                ("edges", ctypes.POINTER(ctypes.c_double))]


class tsb_multipole(ctypes.Structure):
    _fields_ = [("l1", ctypes.c_int32), ("l2", ctypes.c_int32), ("L", ctypes.c_int32)]


class tsb_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("pair_mode", ctypes.c_int32), ("box_mode", ctypes.c_int32),
                ("P0", ctypes.c_double), ("unfused", ctypes.c_int32), ("estimator", ctypes.c_int32),
                ("shot_noise", ctypes.c_int32), ("assign_tiles", ctypes.c_int32)]


class tsb_catalog(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("nbar", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("on_device", ctypes.c_int32)]


class tsb_plan_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("r_f", ctypes.c_int32), ("r_g", ctypes.c_int32),
                ("n_channels", ctypes.c_int32), ("n_fields_f", ctypes.c_int32), ("n_fields_g", ctypes.c_int32),
                ("n_outputs", ctypes.c_int32), ("n_grids", ctypes.c_int32), ("n_fslots", ctypes.c_int32),
                ("fused", ctypes.c_int32), ("n_terms", ctypes.c_int32), ("workspace_bytes", ctypes.c_int64),
                ("reduce_flops", ctypes.c_int64), ("assign_columns", ctypes.c_int32)]


_P = ctypes.POINTER
_lib.tsb_last_error.restype = ctypes.c_char_p
_lib.tsb_last_error.argtypes = []
_lib.tsb_plan_create.restype = ctypes.c_int
_lib.tsb_plan_create.argtypes = [_P(tsb_grid), _P(tsb_los), _P(tsb_kbins), _P(tsb_multipole), ctypes.c_int32,
                                 _P(tsb_options), _P(ctypes.c_void_p)]
_lib.tsb_request_query.restype = ctypes.c_int
_lib.tsb_request_query.argtypes = [_P(tsb_grid), _P(tsb_los), _P(tsb_kbins), _P(tsb_multipole), ctypes.c_int32,
                                   _P(tsb_options), _P(tsb_plan_info), _P(ctypes.c_int64), _P(ctypes.c_double)]
_lib.tsb_plan_query.restype = ctypes.c_int
_lib.tsb_plan_query.argtypes = [ctypes.c_void_p, _P(ctypes.c_int64), _P(ctypes.c_int64), _P(ctypes.c_int64)]
_lib.tsb_plan_shot_noise.restype = ctypes.c_int
_lib.tsb_plan_shot_noise.argtypes = [ctypes.c_void_p, _P(ctypes.c_double), _P(ctypes.c_double)]
_lib.tsb_plan_destroy.restype = ctypes.c_int
_lib.tsb_plan_destroy.argtypes = [ctypes.c_void_p]
_lib.tsb_plan_get_info.restype = ctypes.c_int
_lib.tsb_plan_get_info.argtypes = [ctypes.c_void_p, _P(tsb_plan_info)]
_lib.tsb_plan_nmode.restype = ctypes.c_int
_lib.tsb_plan_nmode.argtypes = [ctypes.c_void_p, _P(ctypes.c_int64), _P(ctypes.c_double)]
_lib.tsb_plan_channel.restype = ctypes.c_int
_lib.tsb_plan_channel.argtypes = [ctypes.c_void_p, ctypes.c_int32, _P(ctypes.c_int32), _P(ctypes.c_int32),
                                  _P(ctypes.c_int32)]
_lib.tsb_measure.restype = ctypes.c_int
_lib.tsb_measure.argtypes = [ctypes.c_void_p, _P(tsb_catalog), _P(tsb_catalog), ctypes.c_void_p,
                             _P(ctypes.c_double), _P(ctypes.c_double), _P(ctypes.c_double)]
_lib.tsb_measure_noalloc.restype = ctypes.c_int
_lib.tsb_measure_noalloc.argtypes = [ctypes.c_void_p, _P(tsb_catalog), _P(tsb_catalog), ctypes.c_void_p,
                                     _P(ctypes.c_double), _P(ctypes.c_double), _P(ctypes.c_double)]
_lib.tsb_assign.restype = ctypes.c_int
_lib.tsb_assign.argtypes = [ctypes.c_void_p, _P(tsb_catalog), _P(tsb_catalog), ctypes.c_void_p, ctypes.c_void_p]

_lib.tsb_plan_set_profiling.restype = ctypes.c_int
_lib.tsb_plan_set_profiling.argtypes = [ctypes.c_void_p, ctypes.c_int32]
_lib.tsb_plan_autotune.restype = ctypes.c_int
_lib.tsb_plan_autotune.argtypes = [ctypes.c_void_p, _P(tsb_catalog), _P(tsb_catalog), ctypes.c_void_p, ctypes.c_int32,
                                   _P(ctypes.c_int32)]
_lib.tsb_plan_stage_times.restype = ctypes.c_int
_lib.tsb_plan_stage_times.argtypes = [ctypes.c_void_p, ctypes.c_int32, _P(ctypes.c_double), _P(ctypes.c_int64),
                                      ctypes.c_int32]

_lib.tsb_measure_batch.restype = ctypes.c_int
_lib.tsb_measure_batch.argtypes = [_P(ctypes.c_void_p), _P(_P(tsb_catalog)), _P(_P(tsb_catalog)), ctypes.c_int32,
                                   ctypes.c_void_p, _P(_P(ctypes.c_double)), _P(ctypes.c_double),
                                   _P(ctypes.c_double)]
_lib.tsb_wigner_9j.restype = ctypes.c_int
_lib.tsb_wigner_9j.argtypes = [_P(ctypes.c_int32), _P(ctypes.c_double)]
_lib.tsb_masked_zeta.restype = ctypes.c_int
_lib.tsb_masked_zeta.argtypes = [_P(tsb_multipole), ctypes.c_int32, ctypes.c_void_p, _P(tsb_multipole), ctypes.c_int32,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                 _P(tsb_multipole), ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                 _P(ctypes.c_double)]
_lib.tsb_masked_bispectrum.restype = ctypes.c_int
_lib.tsb_masked_bispectrum.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_void_p]
_lib.tsb_plan_set_schedule.restype = ctypes.c_int
_lib.tsb_plan_set_schedule.argtypes = [ctypes.c_void_p, _P(ctypes.c_int32)]
_lib.tsb_plan_set_graphs.restype = ctypes.c_int
_lib.tsb_plan_set_graphs.argtypes = [ctypes.c_void_p, ctypes.c_int32]
_lib.tsb_server_create.restype = ctypes.c_int
_lib.tsb_server_create.argtypes = [ctypes.c_int64, ctypes.c_int32, _P(ctypes.c_void_p)]
_lib.tsb_server_submit.restype = ctypes.c_int
_lib.tsb_server_submit.argtypes = [ctypes.c_void_p, ctypes.c_void_p, _P(tsb_catalog), _P(tsb_catalog),
                                   _P(ctypes.c_double), _P(ctypes.c_int64)]
_lib.tsb_server_poll.restype = ctypes.c_int
_lib.tsb_server_poll.argtypes = [ctypes.c_void_p, ctypes.c_int64, _P(ctypes.c_int32), _P(ctypes.c_double)]
_lib.tsb_server_wait.restype = ctypes.c_int
_lib.tsb_server_wait.argtypes = [ctypes.c_void_p, ctypes.c_int64, _P(ctypes.c_double)]
_lib.tsb_server_stats.restype = ctypes.c_int
_lib.tsb_server_stats.argtypes = [ctypes.c_void_p, _P(ctypes.c_int32), _P(ctypes.c_int64)]
_lib.tsb_server_destroy.restype = ctypes.c_int
_lib.tsb_server_destroy.argtypes = [ctypes.c_void_p]

STAGES = ["weights", "bucket", "assign", "fwd_z", "fwd_y", "fwd_x", "combine", "invF_x", "invF_y", "invF_z",
          "invG_x", "invG_y", "invG_z", "reduce", "reduce_final"]

EXPORTED = ["tsb_plan_set_profiling", "tsb_plan_stage_times", "tsb_plan_autotune", "tsb_plan_create", "tsb_plan_destroy",
            "tsb_plan_query", "tsb_request_query", "tsb_plan_get_info", "tsb_plan_nmode", "tsb_measure",
            "tsb_measure_noalloc",
            "tsb_plan_shot_noise", "tsb_assign", "tsb_plan_channel", "tsb_last_error", "tsb_measure_batch",
            "tsb_plan_set_graphs", "tsb_plan_set_schedule", "tsb_server_create", "tsb_server_submit", "tsb_server_poll", "tsb_server_wait",
            "tsb_server_stats", "tsb_server_destroy", "tsb_wigner_9j", "tsb_masked_zeta", "tsb_masked_bispectrum"]


def tsb_last_error():
    return _lib.tsb_last_error().decode()


def _check(rc):
    if rc != TSB_OK:
        raise TsbError(rc, tsb_last_error())
    return rc


def tsb_plan_create(grid, los, bins, multipoles, options):
    arr = (tsb_multipole * len(multipoles))(*multipoles)
    h = ctypes.c_void_p()
    _check(_lib.tsb_plan_create(ctypes.byref(grid), ctypes.byref(los), ctypes.byref(bins), arr,
                                len(multipoles), ctypes.byref(options), ctypes.byref(h)))
    return h


def tsb_request_query(grid, los, bins, multipoles, options, n_bins):
    """Host-only validation: (info, nmode list, k_eff list)."""
    arr = (tsb_multipole * len(multipoles))(*multipoles)
    info = tsb_plan_info()
    nm = (ctypes.c_int64 * n_bins)()
    ke = (ctypes.c_double * n_bins)()
    _check(_lib.tsb_request_query(ctypes.byref(grid), ctypes.byref(los), ctypes.byref(bins), arr,
                                  len(multipoles), ctypes.byref(options), ctypes.byref(info), nm, ke))
    return info, list(nm), list(ke)


def tsb_plan_query(h, n_bins):
    """(workspace bytes, computed (multipole, b1, b2) entries, nmode list)."""
    ws, npairs = ctypes.c_int64(), ctypes.c_int64()
    nm = (ctypes.c_int64 * n_bins)()
    _check(_lib.tsb_plan_query(h, ctypes.byref(ws), ctypes.byref(npairs), nm))
    return ws.value, npairs.value, list(nm)


def tsb_plan_shot_noise(h, S_ptr, S_ijk_ptr=None):
    return _check(_lib.tsb_plan_shot_noise(h, ctypes.cast(S_ptr, _P(ctypes.c_double)),
                                           None if S_ijk_ptr is None else ctypes.cast(S_ijk_ptr, _P(ctypes.c_double))))


def tsb_plan_destroy(h):
    return _check(_lib.tsb_plan_destroy(h))


def tsb_plan_get_info(h):
    info = tsb_plan_info()
    _check(_lib.tsb_plan_get_info(h, ctypes.byref(info)))
    return info


def tsb_plan_nmode(h, n_bins):
    nm = (ctypes.c_int64 * n_bins)()
    ke = (ctypes.c_double * n_bins)()
    _check(_lib.tsb_plan_nmode(h, nm, ke))
    return list(nm), list(ke)


def tsb_plan_channel(h, c):
    L, M, part = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.tsb_plan_channel(h, c, ctypes.byref(L), ctypes.byref(M), ctypes.byref(part)))
    return L.value, M.value, part.value


def tsb_measure(h, data, randoms, stream, B_out_ptr):
    """data / randoms: tsb_catalog (randoms may be None); B_out_ptr: pointer to a
    host double buffer. Returns (I, alpha)."""
    I = ctypes.c_double()
    alpha = ctypes.c_double()
    _check(_lib.tsb_measure(h, ctypes.byref(data), ctypes.byref(randoms) if randoms is not None else None,
                            stream, ctypes.cast(B_out_ptr, _P(ctypes.c_double)), ctypes.byref(I),
                            ctypes.byref(alpha)))
    return I.value, alpha.value


def tsb_measure_noalloc(h, data, randoms, stream, B_out_ptr):
    """As tsb_measure, in the library's static scratch. Returns (I, alpha)."""
    I = ctypes.c_double()
    alpha = ctypes.c_double()
    _check(_lib.tsb_measure_noalloc(h, ctypes.byref(data), ctypes.byref(randoms) if randoms is not None else None,
                                    stream, ctypes.cast(B_out_ptr, _P(ctypes.c_double)), ctypes.byref(I),
                                    ctypes.byref(alpha)))
    return I.value, alpha.value


def tsb_assign(h, data, randoms, stream, grids_out_ptr):
    return _check(_lib.tsb_assign(h, ctypes.byref(data), ctypes.byref(randoms) if randoms is not None else None,
                                  stream, grids_out_ptr))


def tsb_plan_set_profiling(h, stages=True):
    """stages: True (every stage), False/None (off) or an iterable of stage names."""
    if stages is True:
        mask = -1
    elif not stages:
        mask = 0
    else:
        mask = 0
        for name in stages:
            mask |= 1 << STAGES.index(name)
    return _check(_lib.tsb_plan_set_profiling(h, mask))


def tsb_plan_autotune(h, data, randoms, stream, reps=3):
    """Tune the plan's launch schedule; returns {stage: lines per workgroup
    (0 = LDS rule)} for the tuned FFT stages, 'tile_wgs', 'reduce_row_tasks'
    (1 row tasks, 0 shell tasks, 2 columns then rows, or -1 when the one-pass
    reduction is not used) and 'reduce_block'
    (512, 1024, or -1 when the unfused matrix-core reduction is not used)."""
    choice = (ctypes.c_int32 * 18)()
    _check(_lib.tsb_plan_autotune(h, data, randoms, ctypes.c_void_p(stream), int(reps), choice))
    out = {name: int(choice[i]) for i, name in enumerate(STAGES) if choice[i]}
    out["tile_wgs"] = int(choice[len(STAGES)])
    out["reduce_row_tasks"] = int(choice[len(STAGES) + 1])
    out["reduce_block"] = int(choice[len(STAGES) + 2])
    return out


def tsb_wigner_9j(*l):
    arr = (ctypes.c_int32 * 9)(*[int(v) for v in l])
    out = ctypes.c_double()
    _check(_lib.tsb_wigner_9j(arr, ctypes.byref(out)))
    return out.value


def _mults(ms):
    return (tsb_multipole * len(ms))(*[tsb_multipole(*map(int, m)) for m in ms])


def tsb_masked_zeta(model, zeta_ptr, window, Q_ptr, r_ptr, w_ptr, n_r, out, zeta_out_ptr, integral):
    zbar = ctypes.c_double()
    _check(_lib.tsb_masked_zeta(_mults(model), len(model), zeta_ptr, _mults(window), len(window), Q_ptr, r_ptr,
                                w_ptr, int(n_r), _mults(out), len(out), int(bool(integral)), zeta_out_ptr,
                                ctypes.byref(zbar)))
    return zbar.value


def tsb_masked_bispectrum(l1, l2, zeta_ptr, r_ptr, w_ptr, n_r, k_ptr, n_k, B_ptr):
    _check(_lib.tsb_masked_bispectrum(int(l1), int(l2), zeta_ptr, r_ptr, w_ptr, int(n_r), k_ptr, int(n_k), B_ptr))


def tsb_plan_set_schedule(h, choice):
    """Apply a schedule in the layout tsb_plan_autotune returns (a dict)."""
    arr = (ctypes.c_int32 * 18)()
    for i, name in enumerate(STAGES):
        arr[i] = int(choice.get(name, 0))
    arr[len(STAGES)] = int(choice.get("tile_wgs", 0))
    arr[len(STAGES) + 1] = int(choice.get("reduce_row_tasks", -1))
    arr[len(STAGES) + 2] = int(choice.get("reduce_block", -1))
    _check(_lib.tsb_plan_set_schedule(h, arr))


def tsb_plan_stage_times(h, reset=False):
    """{stage name: (accumulated ms, launches)}"""
    n = len(STAGES)
    ms = (ctypes.c_double * n)()
    calls = (ctypes.c_int64 * n)()
    _check(_lib.tsb_plan_stage_times(h, n, ms, calls, int(bool(reset))))
    return {STAGES[i]: (ms[i], calls[i]) for i in range(n)}


def tsb_measure_batch(handles, datas, randoms, stream, B_ptrs):
    """handles: plan handles; datas / randoms: tsb_catalog structs (randoms None
    or a list with None in box mode); B_ptrs: host double-buffer pointers.
    Returns (I list, alpha list)."""
    n = len(handles)
    hs = (ctypes.c_void_p * n)(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    ds = (_P(tsb_catalog) * n)(*[ctypes.pointer(d) for d in datas])
    rs = None
    if randoms is not None:
        rs = (_P(tsb_catalog) * n)(*[ctypes.pointer(r) if r is not None else None for r in randoms])
    bs = (_P(ctypes.c_double) * n)(*[ctypes.cast(p, _P(ctypes.c_double)) for p in B_ptrs])
    I = (ctypes.c_double * n)()
    alpha = (ctypes.c_double * n)()
    _check(_lib.tsb_measure_batch(hs, ds, rs, n, stream, bs, I, alpha))
    return list(I), list(alpha)


def tsb_plan_set_graphs(h, enable):
    return _check(_lib.tsb_plan_set_graphs(h, int(bool(enable))))


def tsb_server_create(budget_bytes, max_slots):
    h = ctypes.c_void_p()
    _check(_lib.tsb_server_create(int(budget_bytes), int(max_slots), ctypes.byref(h)))
    return h


def tsb_server_submit(srv, plan, data, randoms, B_ptr):
    t = ctypes.c_int64()
    _check(_lib.tsb_server_submit(srv, plan, ctypes.byref(data),
                                  ctypes.byref(randoms) if randoms is not None else None,
                                  ctypes.cast(B_ptr, _P(ctypes.c_double)), ctypes.byref(t)))
    return t.value


def tsb_server_poll(srv, ticket):
    """(done, latency_s); raises the request's error once it is done and failed."""
    done = ctypes.c_int32()
    lat = ctypes.c_double()
    _check(_lib.tsb_server_poll(srv, ticket, ctypes.byref(done), ctypes.byref(lat)))
    return bool(done.value), lat.value


def tsb_server_wait(srv, ticket):
    lat = ctypes.c_double()
    _check(_lib.tsb_server_wait(srv, ticket, ctypes.byref(lat)))
    return lat.value


def tsb_server_stats(srv):
    """(peak requests running at once, workspaces released)."""
    peak, rel = ctypes.c_int32(), ctypes.c_int64()
    _check(_lib.tsb_server_stats(srv, ctypes.byref(peak), ctypes.byref(rel)))
    return peak.value, rel.value


def tsb_server_destroy(srv):
    return _check(_lib.tsb_server_destroy(srv))
