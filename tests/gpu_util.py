"""Shared helpers of the GPU parity tests (input plumbing and comparisons only)."""
import math
import os
import sys

import numpy as np

from oracle import estimator as est


def oracle_plan(**kw):
    """Oracle Plan from the keyword request used by paper_1803_02132_amd.Plan."""
    keep = {k: kw[k] for k in ("n", "box_len", "multipoles", "n_bins", "dk", "k_min", "origin", "assign_p",
                               "interlace", "los", "los_dir", "observer", "box_mode", "P0", "edges", "vertex") if k in kw}
    if keep.get("edges") is not None:
        keep["edges"] = tuple(float(e) for e in keep["edges"])
    keep["interlace"] = bool(keep.get("interlace", False))
    return est.Plan(**keep)


def pair_mask(multipoles, n_bins, pair_mode="paper"):
    m = np.zeros((len(multipoles), n_bins, n_bins), dtype=bool)
    for mu, (l1, l2, L) in enumerate(multipoles):
        for b1 in range(n_bins):
            for b2 in range(n_bins):
                if pair_mode == "paper":
                    m[mu, b1, b2] = (b1 <= b2) if l1 == l2 else True
                elif pair_mode == "upper":
                    m[mu, b1, b2] = b1 <= b2
                elif pair_mode == "diagonal":
                    m[mu, b1, b2] = b1 == b2
                else:
                    m[mu, b1, b2] = True
    return m


def normwise_errors(B_gpu, B_or, mask):
    """Per multipole: max |dB| / max |B_oracle| over the computed pairs."""
    out = []
    for mu in range(B_or.shape[0]):
        sel = mask[mu]
        ref = np.max(np.abs(B_or[mu][sel]))
        err = np.max(np.abs(B_gpu[mu][sel] - B_or[mu][sel]))
        out.append(err / ref if ref > 0 else err)
    return np.array(out)


def box_request(n=32, box_len=1000.0, n_bins=8, dk=None, **kw):
    if dk is None:
        dk = 2.0 * 2.0 * math.pi / box_len
    req = dict(n=n, box_len=box_len, n_bins=n_bins, dk=dk, k_min=0.0, multipoles=[(0, 0, 0), (2, 0, 2)],
               assign_p=3, interlace=True, los="local", observer=(box_len / 2, box_len / 2, -1.5 * box_len),
               box_mode=True, precision="f32")
    req.update(kw)
    return req


# Lines printed by the GPU tests (errors against the oracle per multipole and
# the like), repeated in the run's terminal summary by conftest.py.
REPORT = []


def report(*a):
    """Print a result line and keep it, with the test's id, for the summary."""
    def fmt(x):
        if isinstance(x, np.ndarray) and x.dtype.kind == "f":
            return np.array2string(x, formatter={"float_kind": lambda v: f"{v:.2e}"})
        if isinstance(x, float):
            return f"{x:.6g}"
        return str(x)
    line = " ".join(fmt(x) for x in a)
    print(line, flush=True)
    sys.stdout.flush()
    test = os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0].split("::")[-1]
    REPORT.append(f"{test}: {line}" if test else line)
