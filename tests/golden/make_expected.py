"""Write the oracle's expected multipoles for the full-size GPU parity tests.

Calls only the FP64 oracle and the seeded mock generator; nothing here comes
from the HIP path. Run from the repository root:
    python tests/golden/make_expected.py
Outputs (small .npz files next to this script):
  box128_seed0.npz   every pair of the 128^3 box workload (500k particles,
                     Kaiser along a local LOS, TSC + interlacing, 000 110 202 112)
  box128_shot_seed0.npz the shot noise of the same measurement (Sec. 4.2,
                     eqs. 44-46): its four terms, S and B - S, every pair
  box256_seed48.npz  every shell pair of one 256^3 throughput mock (000, 202):
                     the configuration the benchmark times
  box512_seed7002.npz sampled shell pairs of a 512^3 request (the largest grid
                     of the serving mix): 2M particles, global LOS along z,
                     000 202
  survey256_seed3.npz shell pairs of the 256^3 survey-window workload that
                     touch every one of its 25 shells (2M galaxies in a half
                     shell, 20M randoms, FKP weights, 000 202 112 404)
  serve384_seed7001.npz sampled shell pairs of a 384^3 serving request
                     (2M particles, 000 110 202)
Pass workload names (box128 box128_shot box256 box512 survey256 serve384) to write only those files.
Each file also stores a checksum of the generated catalogue so the tests can
confirm they regenerated the same input.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from mocks.lognormal import WORKLOADS, survey_workload, workload  # noqa: E402
from oracle import estimator as est  # noqa: E402
from oracle import shotnoise as sn  # noqa: E402

# every shell once as b1 and once as b2: (b, b + 6 mod 25); the upper pairs
# (b1 < b2) alone cover every shell, so the b1 <= b2 multipoles see all of them
SAMPLED_PAIRS_SURVEY = [(b, (b + 6) % 25) for b in range(25)] + [(0, 0), (12, 12), (24, 24)]
SAMPLED_PAIRS_512 = [(0, 0), (2, 17), (5, 5), (7, 12), (9, 14), (14, 9), (19, 19)]
SAMPLED_PAIRS_384 = [(4, 4), (4, 15), (15, 4), (15, 15)]


def catalogue_checksum(cat):
    p = np.asarray(cat["pos"], np.float64)
    return np.array([len(p), p.sum(), (p * p).sum()])


def oracle_plan(spec, box_mode=True):
    return est.Plan(n=spec["n"], box_len=spec["box_len"], multipoles=spec["multipoles"], n_bins=spec["n_bins"],
                    dk=spec["dk"], k_min=spec["k_min"], assign_p=spec["assign_p"], interlace=spec["interlace"],
                    los=spec["los"], observer=spec.get("observer", (0.0, 0.0, 0.0)), box_mode=box_mode,
                    P0=spec.get("P0", 0.0))


def measure_lean(plan, data, randoms=None, pairs=None):
    """est.measure without keeping the assigned grids (full-size grids)."""
    grids, info = est.assign_channels(plan, data, randoms)
    spec = est.spectra(plan, grids)
    del grids
    Bre, Bim = est.reduce_fft(plan, spec, info["I"], pairs=pairs)
    return {"B": Bre, "B_imag": Bim, "I": info["I"], "alpha": info["alpha"], "nmode": est.nmode(plan)}


def survey256():
    t0 = time.time()
    spec, data, rand = survey_workload("survey256", seed=3)
    res = measure_lean(oracle_plan(spec, box_mode=False), data, rand, pairs=SAMPLED_PAIRS_SURVEY)
    np.savez(os.path.join(HERE, "survey256_seed3.npz"), B=res["B"], B_imag=res["B_imag"], I=res["I"],
             alpha=res["alpha"], nmode=res["nmode"], pairs=np.array(SAMPLED_PAIRS_SURVEY),
             checksum=catalogue_checksum(data), checksum_randoms=catalogue_checksum(rand))
    print(f"survey256 done in {time.time() - t0:.0f} s", flush=True)


def box128():
    t0 = time.time()
    spec, cat = workload("box128", seed=0)
    res = est.measure(oracle_plan(spec), cat)
    np.savez(os.path.join(HERE, "box128_seed0.npz"), B=res["B"], B_imag=res["B_imag"], I=res["I"],
             nmode=res["nmode"], checksum=catalogue_checksum(cat))
    print(f"box128 done in {time.time() - t0:.0f} s", flush=True)


def box128_shot():
    t0 = time.time()
    spec, cat = workload("box128", seed=0)
    res = sn.measure_shot_noise(oracle_plan(spec), cat)
    np.savez(os.path.join(HERE, "box128_shot_seed0.npz"), B=res["B"], S=res["S"], S_iii=res["iii"],
             S_ij=res["ij"], S_jk=res["jk"], S_ik=res["ik"], I=res["I"], checksum=catalogue_checksum(cat))
    print(f"box128_shot done in {time.time() - t0:.0f} s", flush=True)


def box256():
    t0 = time.time()
    spec, cat = workload("box256", seed=48)
    res = measure_lean(oracle_plan(spec), cat)
    np.savez(os.path.join(HERE, "box256_seed48.npz"), B=res["B"], B_imag=res["B_imag"], I=res["I"],
             nmode=res["nmode"], checksum=catalogue_checksum(cat))
    print(f"box256 done in {time.time() - t0:.0f} s", flush=True)


def box512():
    # the largest grid of the serving mix: 2M particles of a mock whose field
    # lives on a 256^3 grid, measured on 512^3 with a global LOS along z
    # (one assigned channel, so the oracle's grids fit in host memory)
    t0 = time.time()
    spec, cat = workload("box256", seed=7002, n_target=2_000_000)
    spec = dict(spec, n=512, multipoles=[(0, 0, 0), (2, 0, 2)], los="global")
    res = measure_lean(oracle_plan(spec), cat, pairs=SAMPLED_PAIRS_512)
    np.savez(os.path.join(HERE, "box512_seed7002.npz"), B=res["B"], B_imag=res["B_imag"], I=res["I"],
             nmode=res["nmode"], pairs=np.array(SAMPLED_PAIRS_512), checksum=catalogue_checksum(cat))
    print(f"box512 done in {time.time() - t0:.0f} s", flush=True)


def serve384():
    # a serving request on a radix-3 grid: 2M particles of a mock whose field
    # lives on a 256^3 grid, measured on 384^3 with {000, 110, 202}
    t0 = time.time()
    spec, cat = workload("box256", seed=7001, n_target=2_000_000)
    spec = dict(spec, n=384, multipoles=[(0, 0, 0), (1, 1, 0), (2, 0, 2)])
    res = measure_lean(oracle_plan(spec), cat, pairs=SAMPLED_PAIRS_384)
    np.savez(os.path.join(HERE, "serve384_seed7001.npz"), B=res["B"], B_imag=res["B_imag"], I=res["I"],
             nmode=res["nmode"], pairs=np.array(SAMPLED_PAIRS_384), checksum=catalogue_checksum(cat))
    print(f"serve384 done in {time.time() - t0:.0f} s", flush=True)


TARGETS = {"box128": box128, "box128_shot": box128_shot, "box256": box256, "box512": box512, "survey256": survey256, "serve384": serve384}


if __name__ == "__main__":
    for name in sys.argv[1:] or list(TARGETS):
        TARGETS[name]()
