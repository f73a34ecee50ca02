"""Throughput of the bispectrum-multipole hot path on one MI355X.

One step = one full measurement (weights, y-weighted TSC+interlaced assignment,
forward FFTs, shell filters, inverse FFTs, 3j-weighted reduction, normalisation)
of one 256^3 mock, with its catalogue already resident in HBM:
  box L = 1000 Mpc/h, 256^3 grid, TSC + interlacing, local LOS from an observer
  1500 Mpc/h below the box centre, 20 shells of dk = 0.01 h/Mpc from 0,
  B_000 (210 pairs k1 <= k2) and B_202 (400 pairs), particles log-uniform in
  [3e5, 3e6] (seeded lognormal + Kaiser mocks; steps cycle over the mocks).

Prints one JSON line with throughput (mocks/s), the roofline of the dominant
kernel (algorithmic bytes per launch / its mean duration from HIP events on the
launch stream over the timed region) and the FP64 oracle timed on a bounded
sample on the host. The per-stage table (`stage_ms`) comes from a pass with
events around every stage, run before the timed region; inside it only the
dominant stage carries events.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = dict(n=256, box_len=1000.0, n_bins=20, dk=0.01, k_min=0.0, multipoles=[(0, 0, 0), (2, 0, 2)],
                assign_p=3, interlace=True, los="local", observer=(500.0, 500.0, -1000.0), box_mode=True,
                precision="f32", pair_mode="paper")
SEEDS = [48, 49, 50, 51]
KERNEL_SOURCES = {  # which source file holds each stage's kernel
    "assign": "assign.hip", "fwd_z": "fft.hip", "fwd_y": "fft.hip", "fwd_x": "fft.hip",
    "invF_x": "fft.hip", "invF_y": "fft.hip", "invF_z": "fft.hip", "invG_x": "fft.hip",
    "invG_y": "fft.hip", "invG_z": "fft.hip", "reduce": "fused.hip"}


FP32_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload_request(name):
    """The plan request of a named workload (the throughput mock, the 128^3
    box, the 256^3 survey window)."""
    if name == "box256":
        return dict(WORKLOAD)
    from mocks.lognormal import WORKLOADS
    w = WORKLOADS[name]
    req = dict(n=w["n"], box_len=w["box_len"], n_bins=w["n_bins"], dk=w["dk"], k_min=w["k_min"],
               multipoles=w["multipoles"], assign_p=w["assign_p"], interlace=w["interlace"], los=w["los"],
               observer=w["observer"], box_mode=True, precision=w["precision"], pair_mode="paper")
    if name == "survey256":
        req.update(box_mode=False, P0=w["P0"])
    return req


def live_lines(r, r2):
    """Lines of a pruned cube (frequencies |n_i| <= r) that the inverse chain
    reads or writes under the sparsity rule (zero beyond |n|^2 = r2): the
    (n_a, n_b) pairs of the x pass and the n_b values of the y pass."""
    f = np.arange(-r, r + 1)
    return int(np.sum(f[:, None] ** 2 + f[None, :] ** 2 <= r2)), int(np.sum(f * f <= r2))


def shell_r2(info, req):
    """Largest |n|^2 of the modes of each k-shell (the library's bin rule)."""
    kf = 2.0 * math.pi / req["box_len"]
    n2 = np.arange(3 * info.r_f ** 2 + 1)
    b = np.floor((kf * np.sqrt(n2) - req["k_min"]) / req["dk"]).astype(np.int64)
    return [int(n2[b == i].max()) if np.any(b == i) else -1 for i in range(req["n_bins"])]


def stage_bytes(info, copies, n_particles, req, fused=True, esz=4):
    """Algorithmic HBM bytes per launch of each single-kernel stage: every input
    read once and every output written once in the stated layout (particle
    records: 12 B of position plus 4 B per channel). A plan that assigns by
    columns writes the z pass's output from the assignment (the grids are
    never stored), so its assign stage holds the records and that output and
    it has no fwd_z stage. The inverse transforms of
    shell-filtered and band-limited spectra count the lines and entries that
    can be non-zero: for shell b, the (n_y, n_z) lines of the x pass and the
    n_z entries after it with |n|^2 within the shell's largest |n|^2."""
    c = 2 * esz
    N, M = info.n, info.m
    PG, PF = 2 * info.r_g + 1, 2 * info.r_f + 1
    ng = info.n_grids
    nbc = copies * ng
    nk = info.n_fslots
    nf = nk * req["n_bins"]
    lf = [live_lines(info.r_f, r2) for r2 in shell_r2(info, req)]
    lf1 = nk * sum(x[0] for x in lf)       # live x-pass lines over every F slot
    lf2 = nk * sum(x[1] for x in lf)       # live y-pass lines per x over every F slot
    if 4 * info.r_f < info.n:   # band-limited G (the reduced-grid rule): |n|^2 <= 4 n2max of the shells
        g1, g2 = live_lines(info.r_g, 4 * max(shell_r2(info, req)))
    else:
        g1, g2 = PG * PG, PG
    out = {
        "assign": nbc * N ** 3 * c + (24 + 4 * info.n_channels) * n_particles,
        "fwd_z": nbc * N ** 3 * c + nbc * N * N * PG * c,
        "fwd_y": nbc * N * N * PG * c + nbc * N * PG * PG * c,
        "fwd_x": nbc * N * PG * PG * c + nbc * PG ** 3 * c,
        "invF_x": PF ** 3 * c + lf1 * M * c,
        "invF_y": lf1 * M * c + lf2 * M * M * c,
        "invG_x": ng * PG ** 3 * c + ng * M * g1 * c,
        "invG_y": ng * M * g1 * c + ng * M * M * g2 * c,
        "invG_z": ng * M * M * g2 * c + ng * M ** 3 * c,
    }
    if getattr(info, "assign_columns", 0):
        out["assign"] = nbc * N * N * PG * c + (24 + 4 * info.n_channels) * n_particles
        del out["fwd_z"]
    if fused:   # last F transform inside the reduction: reads the y-pass output and G
        out["reduce"] = lf2 * M * M * c + ng * M ** 3 * c
    else:
        out["invF_z"] = lf2 * M * M * c + nf * M ** 3 * c
        out["reduce"] = (nf + ng) * M ** 3 * c
    return out


def source_hash(fname):
    with open(os.path.join(ROOT, "paper_1803_02132_amd", "csrc", fname), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def plan_geometry(info, req):
    """The plan shape a set of byte counters belongs to."""
    return {"n": info.n, "m": info.m, "r_f": info.r_f, "r_g": info.r_g, "n_bins": int(req["n_bins"]),
            "n_outputs": info.n_outputs, "n_grids": info.n_grids, "n_fslots": info.n_fslots,
            "copies": 1 + int(bool(req.get("interlace", False))), "box_mode": bool(req.get("box_mode", True)),
            "multipoles": ["".join(map(str, m)) for m in req["multipoles"]]}


def load_traffic(workload, geometry, stage):
    """HBM bytes per launch of `stage` from the committed rocprofv3 counter
    summary of this workload, if it was taken on the same plan geometry and the
    current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("workload") != workload or rec.get("geometry") != geometry:
        return None
    st = rec.get("stages", {}).get(stage)
    if not st or st.get("source_sha256_16") != source_hash(KERNEL_SOURCES[stage]):
        return None
    return st.get("hbm_bytes_per_launch")


COPY_PROBE_BYTES = 512 << 20
# stage -> kernels whose dispatches make up one launch of the stage
STAGE_KERNELS = {"assign": ("tile_parts_kernel", "assign_tile_kernel", "heavy_final_kernel", "zcol_kernel"),
                 "reduce": ("fz_reduce_wide_kernel", "fz_reduce_kernel", "reduce_kernel", "reduce_mfma_kernel",
                            "reduce_mfma_wide_kernel")}
# kernels of the FFT passes (the fused forward x pass with the combination included)
FFT_KERNELS = ("fft4_kernel", "fft4_combine_kernel", "fft_pass_kernel")
# order of the FFT-pass dispatches inside one measurement (fused plan)
FFT_ORDER = ["fwd_z", "fwd_y", "fwd_x", "invG_x", "invG_y", "invG_z", "invF_x", "invF_y"]


def copy_probe(reps=3):
    """A plain device-to-device copy of COPY_PROBE_BYTES, whose HBM byte counters
    calibrate those of the path's kernels (read and write once each)."""
    import torch
    src = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy probe: {reps} x {COPY_PROBE_BYTES} B device-to-device")


def _read_counters(path):
    import csv
    rows = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            d = int(r["Dispatch_Id"])
            rows.setdefault(d, [r["Kernel_Name"], 0.0])
            rows[d][1] += float(r["Counter_Value"])
    return [(d, rows[d][0], rows[d][1]) for d in sorted(rows)]


def ingest_pmc(fetch_csv, write_csv, command, workload="box256"):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per
    dispatch) of `bench.py --copy-probe --workload W` into
    profiles/traffic_W.json (and a .md table): HBM bytes per launch of each
    stage, each counter divided by what it reads for the copy probe relative to
    the probe's true bytes, keyed by the workload and its plan geometry."""
    import paper_1803_02132_amd as tsb
    req = workload_request(workload)
    info = tsb.query(**req)[0]
    geometry = plan_geometry(info, req)
    fused = bool(info.fused)
    order = [st for st in FFT_ORDER if st != "fwd_z" or not info.assign_columns] + ([] if fused else ["invF_z"])
    out = {}
    for label, path in (("fetch", fetch_csv), ("write", write_csv)):
        disp = _read_counters(path)
        probe = [v for (_, k, v) in disp if "copyBuffer" in k and v * 1024 > 0.5 * COPY_PROBE_BYTES]
        if not probe:
            raise SystemExit(f"no copy-probe dispatch in {path}")
        factor = (sum(probe) / len(probe)) * 1024 / COPY_PROBE_BYTES
        starts = [i for i, (_, k, _) in enumerate(disp) if "prep_kernel" in k]
        per = {}
        n_meas = len(starts)
        for j, s0 in enumerate(starts):
            s1 = starts[j + 1] if j + 1 < len(starts) else len(disp)
            ffts = [v for (_, k, v) in disp[s0:s1] if any(n in k for n in FFT_KERNELS)]
            for name, v in zip(order, ffts):
                per[name] = per.get(name, 0.0) + v
            for stage, names in STAGE_KERNELS.items():
                per[stage] = per.get(stage, 0.0) + sum(v for (_, k, v) in disp[s0:s1] if any(n in k for n in names))
        out[label] = {st: (v / n_meas) * 1024 / factor for st, v in per.items()}
        out[label + "_factor"] = factor
    stages = {}
    for st in out["fetch"]:
        f, w = out["fetch"][st], out["write"].get(st, 0.0)
        src = KERNEL_SOURCES.get(st)
        stages[st] = {"fetch_bytes_per_launch": round(f), "write_bytes_per_launch": round(w),
                      "hbm_bytes_per_launch": round(f + w), "source_sha256_16": source_hash(src) if src else None}
    rec = {"workload": workload, "geometry": geometry, "stages": stages,
           "calibration": {"copy_probe_bytes": COPY_PROBE_BYTES, "fetch_counter_per_true_byte": out["fetch_factor"],
                           "write_counter_per_true_byte": out["write_factor"]},
           "command": command}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"traffic_{workload}.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    lines = [f"# HBM traffic per stage launch: {workload}", "", "Command:", "", "    " + command, "",
             f"Plan geometry: {json.dumps(geometry)}", "",
             f"Calibration: a {COPY_PROBE_BYTES} B device copy reads FETCH_SIZE x {out['fetch_factor']:.3f} and "
             f"WRITE_SIZE x {out['write_factor']:.3f} of its true bytes; counts below are divided by these.", "",
             "| stage | fetch (MB) | write (MB) | total (MB) |", "|---|---|---|---|"]
    for st, v in stages.items():
        lines.append(f"| {st} | {v['fetch_bytes_per_launch'] / 1e6:.1f} | {v['write_bytes_per_launch'] / 1e6:.1f} | "
                     f"{v['hbm_bytes_per_launch'] / 1e6:.1f} |")
    with open(os.path.join(ROOT, "profiles", f"traffic_{workload}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


SQ_KERNELS = (("zcol_kernel", "assign by columns + z pass"), ("assign_tile_kernel", "assign"),
              ("fz_reduce_wide_kernel", "reduce (one pass)"),
              ("fz_reduce_kernel", "reduce (one pass, general)"), ("reduce_mfma_wide_kernel", "reduce (matrix cores)"),
              ("fft4_combine_kernel", "fwd_x + combination"), ("fft4_kernel", "FFT passes"),
              ("bucket_fill_kernel", "bucket fill"))


def summarize_sq(csvs, command, out_name, clock_ghz=2.4, simds=1024):
    """Occupancy and issue counters (rocprofv3 --pmc SQ_* runs) per kernel: mean
    resident wavefronts per SIMD = 4 SQ_WAVE_CYCLES / (duration x clock x SIMDs)
    (the SQ counts wave cycles in units of 4 clocks), the shares of a wave's
    lifetime with a VALU instruction active (SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES)
    and waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES), instructions per wave, LDS bank
    conflict cycles per LDS instruction and the MFMA-busy share of the SIMDs."""
    import csv
    per = {}   # (kernel label) -> {counter: [values per dispatch]}, durations
    for path in csvs:
        with open(path) as fh:
            for r in csv.DictReader(fh):
                label = next((lab for key, lab in SQ_KERNELS if key + "<" in r["Kernel_Name"]
                              or r["Kernel_Name"].endswith(key)), None)
                if label is None:
                    continue
                d = per.setdefault(label, {"dur": {}, "vgpr": r.get("VGPR_Count"), "lds": r.get("LDS_Block_Size"),
                                           "wg": r.get("Workgroup_Size")})
                d.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
                d["dur"][(path, r["Dispatch_Id"])] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    lines = [f"# Occupancy and issue counters: {out_name}", "", "Command:", "", "    " + command, "",
             "Per dispatch means. Waves/SIMD: mean resident wavefronts per SIMD (4 SQ_WAVE_CYCLES over the "
             f"dispatch's duration x {clock_ghz} GHz x {simds} SIMDs). VALU active and waiting: shares of the "
             "wavefronts' lifetime (SQ_ACTIVE_INST_VALU and SQ_WAIT_ANY over SQ_WAVE_CYCLES). MFMA busy: "
             "SQ_VALU_MFMA_BUSY_CYCLES over the SIMD cycles of the dispatch.", "",
             "| kernel | VGPRs | workgroup | waves/SIMD | VALU active | waiting | VALU instr/wave | LDS instr/wave | "
             "bank-conflict cycles per LDS instr | MFMA busy |",
             "|---|---|---|---|---|---|---|---|---|---|"]

    def mean(d, k):
        v = d.get(k)
        return sum(v) / len(v) if v else float("nan")

    for key, label in SQ_KERNELS:
        d = per.get(label)
        if not d:
            continue
        dur = sum(d["dur"].values()) / len(d["dur"])
        wc, waves = mean(d, "SQ_WAVE_CYCLES"), mean(d, "SQ_WAVES")
        occ = 4 * wc / (dur * clock_ghz * 1e9 * simds)
        valu = mean(d, "SQ_ACTIVE_INST_VALU") / wc
        wait = mean(d, "SQ_WAIT_ANY") / wc
        lds = mean(d, "SQ_INSTS_LDS")
        mfma = mean(d, "SQ_VALU_MFMA_BUSY_CYCLES") / (dur * clock_ghz * 1e9 * simds)
        lines.append(f"| {label} (`{key}`) | {d['vgpr']} | {d['wg']} | {occ:.2f} | {valu:.1%} | {wait:.1%} | "
                     f"{mean(d, 'SQ_INSTS_VALU') / waves:.0f} | {lds / waves:.0f} | "
                     f"{mean(d, 'SQ_LDS_BANK_CONFLICT') / max(lds, 1):.2f} | {mfma:.1%} |")
    path = os.path.join(ROOT, "profiles", out_name + ".md")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_trace(stats_csv, command, out_name, trace_csv=None, timed=0, bench_log=None):
    """A short text summary of a rocprofv3 --kernel-trace --stats run."""
    import csv
    with open(stats_csv) as fh:
        rows = list(csv.DictReader(fh))
    lines = [f"# Kernel statistics: {out_name}", "", "Command:", "", "    " + command, "",
             "| kernel | calls | mean (us) | total (%) |", "|---|---|---|---|"]
    for r in rows:
        name = r["Name"].replace("(anonymous namespace)::", "").replace("tsb::", "").replace("void ", "")
        short = name.split("(")[0]
        lines.append(f"| `{short}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    if trace_csv and timed:
        # the timed region is the run's last `timed` measurements: per stage,
        # the mean duration of each of its kernels over its last dispatches
        with open(trace_csv) as fh:
            disp = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"])
                          for r in csv.DictReader(fh))
        lines += ["", f"Timed region (the last {timed} dispatches of each kernel of a stage, from the kernel trace "
                  "of the same run; compare the stage mean that the run's bench line reports):", "",
                  "| stage | kernel | mean (us) |", "|---|---|---|"]
        for stage, names in STAGE_KERNELS.items():
            total = 0.0
            for nm in names:
                d = [(e - s) / 1e3 for s, e, k in disp if nm in k][-timed:]
                if d:
                    lines.append(f"| {stage} | `{nm}` | {sum(d) / len(d):.1f} |")
                    total += sum(d) / len(d)
            if total:
                lines.append(f"| {stage} | sum | {total:.1f} |")
    if bench_log:
        # the bench line that the profiled run printed (its event-timed stage means)
        with open(bench_log) as fh:
            js = [ln for ln in fh if ln.startswith("{")]
        if js:
            rec = json.loads(js[-1])
            lines += ["", "Bench line of the same run: " + json.dumps({"value": rec.get("value"),
                                                                      "roofline": rec.get("roofline"),
                                                                      "stage_ms": rec.get("stage_ms")})]
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", out_name + ".md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cat, req, row_pairs=4):
    """The FP64 oracle on a bounded sample of one mock, scaled to one mock, on
    one host thread and on every host thread.

    The oracle evaluates B row by row (one shell b1 at a time, every b2 of the
    row, every multipole). Timed: the front end (weights, every channel's
    assignment, FFTs, deconvolution) on the whole mock; one G field; and one
    row of `row_pairs` shell pairs (its G fields, its b1 F fields, the b2 F
    fields and the products), once with a b2 list of one and once with
    `row_pairs`, which separates a pair's cost from the row's fixed cost.
    One mock = front + every G field + n_bins rows of n_bins pairs. NumPy's
    assignment (bincount) and FFTs run on one thread in both modes (the front
    end is timed once); the multi-threaded mode gives the BLAS products every
    host thread."""
    from threadpoolctl import threadpool_limits
    from oracle import angular as ang
    from oracle import estimator as est
    plan = est.Plan(**{k: req[k] for k in ("n", "box_len", "multipoles", "n_bins", "dk", "k_min", "assign_p",
                                           "los", "observer", "box_mode") if k in req},
                    interlace=bool(req["interlace"]), P0=req.get("P0", 0.0))
    nb = plan.n_bins
    t0 = time.perf_counter()
    grids, info = est.assign_channels(plan, cat)
    spec = est.spectra(plan, grids)
    del grids
    t_front = time.perf_counter() - t0
    log(f"oracle front end: {t_front:.1f} s")
    # distinct G fields the reduction uses
    gset = set()
    for (l1, l2, L) in plan.multipoles:
        for (_, _, M, _) in ang.reduction_terms(l1, l2, L, los="local"):
            if plan.los == "global":
                d = np.asarray(plan.los_dir, np.float64)
                if complex(ang.ylm(L, M, d[0], d[1], d[2])) == 0:
                    continue
            gset.add((L, M))
    t0 = time.perf_counter()
    est.g_field(plan, spec, 0, 0)
    t_g = time.perf_counter() - t0
    b1 = nb // 2
    modes = {}
    for threads in (1, os.cpu_count() or 1):
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            est.reduce_fft(plan, spec, info["I"], pairs=[(b1, 0)])
            t_one = time.perf_counter() - t0
            t0 = time.perf_counter()
            est.reduce_fft(plan, spec, info["I"], pairs=[(b1, b2) for b2 in range(row_pairs)])
            t_row = time.perf_counter() - t0
        t_pair = max((t_row - t_one) / max(row_pairs - 1, 1), 0.0)
        t_fixed = max(t_one - t_pair - len(gset) * t_g, 0.0)   # b1 fields and products
        sec = t_front + len(gset) * t_g + nb * (t_fixed + nb * t_pair)
        log(f"oracle, {threads} thread(s): row fixed {t_fixed:.2f} s, per pair {t_pair:.2f} s, one mock {sec:.0f} s")
        modes[threads] = {"value": 1.0 / sec, "seconds_per_mock": round(sec, 1), "cores": threads,
                          "row_fixed_s": round(t_fixed, 3), "pair_s": round(t_pair, 3)}
    multi = modes[max(modes)]
    return {"value": multi["value"], "unit": "mocks/s", "cores": multi["cores"], "kind": "oracle",
            "cpu_count": os.cpu_count(), "cpu_model": cpu_model(),
            "single_core": modes[1],
            "sample": (f"FP64 NumPy oracle: front end on the whole mock ({t_front:.1f} s, one thread: NumPy "
                       f"bincount and FFT), one G field ({t_g:.2f} s), one row of shell pairs with 1 and "
                       f"{row_pairs} b2 values; one mock = front + {len(gset)} G fields + {nb} rows x {nb} pairs = "
                       f"{multi['seconds_per_mock']:.0f} s on {multi['cores']} threads "
                       f"({modes[1]['seconds_per_mock']:.0f} s on one)")}


# Batched mix (64 mocks of uneven grids): seed s < 24 at 128^3, s < 48 at 192^3,
# else 256^3; particle counts log-uniform in [3e5, 3e6] from the seed.
BATCH_CLASSES = [(128, range(0, 24)), (192, range(24, 48)), (256, range(48, 64))]


def _pool(tsb, sizes, per_size):
    """A pool of distinct seeded catalogues per grid size (device-resident):
    {n: [(seed, n_particles, device catalogue), ...]}."""
    from mocks.lognormal import workload
    pool = {}
    for n, seeds in sizes:
        pool[n] = []
        for s in list(seeds)[:per_size]:
            _, cat = workload("box256", seed=s, n=n)
            pool[n].append((s, len(cat["pos"]), tsb.catalog_to_device(cat)))
            log(f"pool {n}^3 seed {s}: {len(cat['pos'])} particles")
    return pool


def batch_leg(tsb, torch, pool, per_size, replicas=1, autotune=True):
    """64 mocks of mixed grids through tsb_measure_batch, against the same
    measurements made one by one with tsb_measure. Each grid size has
    `replicas` plans (workspaces) that take its items in turn, so that mocks
    of one size also run concurrently."""
    plans = {n: [tsb.Plan(**dict(WORKLOAD, n=n)) for _ in range(replicas)] for n, _ in BATCH_CLASSES}
    items = []
    for n, seeds in BATCH_CLASSES:
        for k, s in enumerate(seeds):
            items.append((plans[n][k % replicas], pool[n][s % per_size][2]))
    ps = [p for p, _ in items]
    ds = [d for _, d in items]
    tuned = {}
    if autotune:                                  # each plan's schedule, on one of its catalogues
        for n, reps in plans.items():
            for p in reps:
                tuned[f"{n}^3"] = p.autotune(pool[n][0][2])
    tsb.measure_batch(ps, ds)                    # warm-up: workspaces, graphs
    for p, d in zip(ps, ds):
        p.measure(d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tsb.measure_batch(ps, ds)
    t_batch = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, d in zip(ps, ds):
        p.measure(d)
    t_plain = time.perf_counter() - t0
    for reps in plans.values():
        for p in reps:
            p.close()
    return {"mocks": len(items), "mix": "24 x 128^3, 24 x 192^3, 16 x 256^3", "plans_per_size": replicas,
            "autotune": tuned or None,
            "distinct_catalogues": sum(len(v) for v in pool.values()),
            "batched_mocks_per_s": round(len(items) / t_batch, 2),
            "plain_mocks_per_s": round(len(items) / t_plain, 2),
            "batched_over_plain": round(t_plain / t_batch, 3)}


def concurrent_leg(tsb, torch, devs, n_plans=3, n_items=48, autotune=True):
    """The headline mocks through tsb_measure_batch with several plans of the
    same geometry, so that consecutive mocks overlap on the device, against the
    same measurements one by one."""
    plans = [tsb.Plan(**WORKLOAD) for _ in range(n_plans)]
    if autotune:
        for p in plans:
            p.autotune(devs[0])
    ps = [plans[i % n_plans] for i in range(n_items)]
    ds = [devs[i % len(devs)] for i in range(n_items)]
    tsb.measure_batch(ps, ds)                    # warm-up: workspaces, graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tsb.measure_batch(ps, ds)
    t_batch = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, d in zip(ps, ds):
        p.measure(d)
    t_plain = time.perf_counter() - t0
    for p in plans:
        p.close()
    return {"plans": n_plans, "mocks": n_items, "batched_mocks_per_s": round(n_items / t_batch, 2),
            "plain_mocks_per_s": round(n_items / t_plain, 2)}


# serving requests: grids, multipoles and particle counts of the request stream
SERVE_SIZES = (128, 192, 256, 384, 512)
SERVE_MULTIPOLES = [(0, 0, 0), (1, 1, 0), (2, 0, 2)]
SERVE_NP = (500_000, 20_000_000)


def serve_catalogue(tsb, seed=7000):
    """One seeded mock of SERVE_NP[1] particles (the headline recipe, field on a
    256^3 grid), shuffled once and resident on the device. A request of N_p
    particles takes the first N_p: a Poisson subsample of the same field."""
    from mocks.lognormal import workload
    _, cat = workload("box256", seed=seed, n_target=SERVE_NP[1])
    perm = np.random.Generator(np.random.PCG64(seed)).permutation(len(cat["pos"]))
    log(f"serving catalogue: {len(perm)} particles")
    return tsb.catalog_to_device({"pos": cat["pos"][perm], "w": None, "nbar": None})


def _prefix(dev, n):
    return {k: (None if v is None else v[:n]) for k, v in dev.items()}


def serve_leg(tsb, torch, big, n_req, rate, slots, budget_gb):
    """Poisson request stream (mean `rate` per second): each request a grid
    drawn uniformly from SERVE_SIZES and N_p log-uniform in SERVE_NP, measuring
    SERVE_MULTIPOLES through the server; then the same requests submitted at
    once (continuous batching under load)."""
    rng = np.random.Generator(np.random.PCG64(2024))
    n_big = int(big["x"].numel())
    tmpl = {n: tsb.Plan(**dict(WORKLOAD, n=n, multipoles=SERVE_MULTIPOLES)) for n in SERVE_SIZES}
    lo, hi = SERVE_NP
    reqs = []
    for _ in range(n_req):
        n = SERVE_SIZES[rng.integers(len(SERVE_SIZES))]
        npart = min(n_big, int(lo * (hi / lo) ** rng.random()))
        reqs.append((n, npart))
    gaps = rng.exponential(1.0 / rate, size=n_req)
    srv = tsb.Server(int(budget_gb * (1 << 30)), slots)
    try:
        for n in SERVE_SIZES:                    # warm-up: a workspace per grid with full particle buffers
            srv.wait(srv.submit(tmpl[n], _prefix(big, n_big)))
        lat, pending = [], {}
        t0 = time.perf_counter()
        t_next = t0
        for k, ((n, npart), gap) in enumerate(zip(reqs, gaps)):
            t_next += gap
            while time.perf_counter() < t_next:
                for t in list(pending):
                    done, l, _ = srv.poll(t)
                    if done:
                        lat.append(l)
                        pending.pop(t)
                time.sleep(0.0005)
            pending[srv.submit(tmpl[n], _prefix(big, npart))] = True
            if (k + 1) % 64 == 0:
                log(f"serving: {k + 1} of {n_req} requests submitted")
        for t in list(pending):
            lat.append(srv.wait(t)[0])
        t_stream = time.perf_counter() - t0
        t0 = time.perf_counter()
        tickets = [srv.submit(tmpl[n], _prefix(big, npart)) for n, npart in reqs]
        lat_burst = [srv.wait(t)[0] for t in tickets]
        t_burst = time.perf_counter() - t0
    finally:
        srv.close()
        for p in tmpl.values():
            p.close()
    ms = np.array(lat) * 1e3
    mb = np.array(lat_burst) * 1e3
    nps = np.array([npart for _, npart in reqs])
    return {"requests": n_req, "rate_per_s": rate, "grids": [f"{n}^3" for n in SERVE_SIZES],
            "multipoles": ["".join(map(str, m)) for m in SERVE_MULTIPOLES],
            "particles": {"min": int(nps.min()), "median": int(np.median(nps)), "max": int(nps.max())},
            "slots": slots, "hbm_budget_gb": budget_gb,
            "poisson": {"mocks_per_s": round(n_req / t_stream, 3), "p50_ms": round(float(np.percentile(ms, 50)), 3),
                        "p99_ms": round(float(np.percentile(ms, 99)), 3)},
            "burst": {"mocks_per_s": round(n_req / t_burst, 2), "p50_ms": round(float(np.percentile(mb, 50)), 3),
                      "p99_ms": round(float(np.percentile(mb, 99)), 3)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--mocks", type=int, default=len(SEEDS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--unfused", action="store_true",
                    help="write the F fields to HBM and reduce in a separate pass (diagnostic)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 64-mock leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--pool", type=int, default=2, help="distinct catalogues per grid size in the batched leg")
    ap.add_argument("--batch-replicas", type=int, default=1, help="plans per grid size in the batched leg")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch schedules (no tsb_plan_autotune before timing)")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=4.0)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-budget-gb", type=float, default=160.0)
    ap.add_argument("--workload", choices=["box256", "box128", "survey256"], default="box256",
                    help="box256: the throughput mock (default, the reported metric); box128 and survey256: "
                         "the 128^3 box and the 256^3 survey-window configurations, for their own timings")
    ap.add_argument("--vertex", choices=["x3", "x1", "x2"], default="x3",
                    help="local LOS at the third vertex (the paper's main text), the first or the second (App. B)")
    ap.add_argument("--pairs", choices=["paper", "diagonal"], default="paper",
                    help="shell pairs measured: the paper's set (default, the reported metric) or the diagonal "
                         "k1 = k2 only (the cheaper measurement of Sec. 4.4), for its own timing")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a device copy of known size (calibrates HBM byte counters)")
    ap.add_argument("--ingest-pmc", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "COMMAND"),
                    help="write profiles/traffic_<workload>.json from two rocprofv3 --pmc runs of "
                         "`bench.py --copy-probe --workload <workload>` and exit")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("STATS_CSV", "COMMAND", "NAME"),
                    help="write profiles/NAME.md from a rocprofv3 kernel-stats CSV and exit")
    ap.add_argument("--summarize-sq", nargs=4, metavar=("CSV1", "CSV2", "COMMAND", "NAME"),
                    help="write profiles/NAME.md from two rocprofv3 --pmc SQ_* counter runs (occupancy, VALU "
                         "activity, waits, LDS conflicts, MFMA busy per kernel)")
    ap.add_argument("--trace-csv", default=None,
                    help="with --summarize-trace: the run's kernel-trace CSV, for the timed-region table")
    ap.add_argument("--timed-launches", type=int, default=0,
                    help="with --trace-csv: measurements in the run's timed region")
    ap.add_argument("--bench-log", default=None,
                    help="with --summarize-trace: the profiled run's output, whose bench line is quoted")
    args = ap.parse_args()
    if args.ingest_pmc:
        ingest_pmc(*args.ingest_pmc, workload=args.workload)
        return
    if args.summarize_sq:
        summarize_sq(args.summarize_sq[:2], args.summarize_sq[2], args.summarize_sq[3])
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace, trace_csv=args.trace_csv, timed=args.timed_launches,
                        bench_log=args.bench_log)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path shards by mock "
              "across GPUs without communication (one plan and request queue per GPU)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1803_02132_amd as tsb
    from mocks.lognormal import workload

    torch.cuda.set_device(0)
    seeds = SEEDS[:max(1, args.mocks)]
    cats, devs = [], []
    req, rands = workload_request(args.workload), None
    if args.workload == "box256":
        for s in seeds:
            spec, cat = workload("box256", seed=s)
            cats.append(cat)
            devs.append(tsb.catalog_to_device(cat))
            log(f"mock seed {s}: {len(cat['pos'])} particles")
    else:
        from mocks.lognormal import survey_workload
        seeds = seeds[:1]
        if args.workload == "survey256":
            spec, cat, rcat = survey_workload("survey256", seed=3)
            rands = [tsb.catalog_to_device(rcat)]
            log(f"survey: {len(cat['pos'])} galaxies, {len(rcat['pos'])} randoms")
        else:
            spec, cat = workload(args.workload, seed=seeds[0])
        cats.append(cat)
        devs.append(tsb.catalog_to_device(cat))
    if args.pairs != "paper":
        req["pair_mode"] = args.pairs
    if args.vertex != "x3":
        req["vertex"] = args.vertex
    plan = tsb.Plan(**dict(req, unfused=args.unfused))

    def step(i):
        k = i % len(devs)
        plan.measure(devs[k], None if rands is None else rands[k])
    info = plan.info
    log(f"plan: N={info.n} M={info.m} r_f={info.r_f} r_g={info.r_g} outputs={info.n_outputs} "
        f"workspace={info.workspace_bytes / 1e9:.2f} GB")
    if args.copy_probe:
        copy_probe()
    tune = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        tune = plan.autotune(devs[0], None if rands is None else rands[0])
        log(f"autotune ({time.perf_counter() - t0:.2f} s): {tune}")
    # Every stage timed with HIP events (they ride inside the captured graph)
    # over the warm-up steps plus one pass over the mocks, outside the timed
    # region: the stage table, and which single-kernel stage dominates.
    tsb.abi.tsb_plan_set_profiling(plan.handle, True)
    for i in range(args.warmup):
        step(i)
    tsb.abi.tsb_plan_stage_times(plan.handle, reset=True)
    for i in range(max(len(devs), 4)):
        step(i)
    times = tsb.abi.tsb_plan_stage_times(plan.handle, reset=True)
    n_mean = float(np.mean([len(c["pos"]) for c in cats]))
    if rands is not None:
        n_mean += float(rands[0]["x"].numel())
    fused = times["invF_z"][1] == 0
    bytes_alg = stage_bytes(info, 1 + int(bool(req["interlace"])), n_mean, req, fused=fused)
    per_launch = {k: (ms / calls if calls else 0.0) for k, (ms, calls) in times.items()}
    log("stage mean ms per launch: " + ", ".join(f"{k}={v:.3f}" for k, v in per_launch.items()))
    dom = max((k for k in bytes_alg), key=lambda k: times[k][0])
    # the timed region keeps events around the dominant stage only (each
    # event pair adds a little time to a measurement)
    tsb.abi.tsb_plan_set_profiling(plan.handle, [dom])
    step(0)                                      # the graph with the new event set
    tsb.abi.tsb_plan_stage_times(plan.handle, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = args.steps / elapsed
    dom_ms, dom_calls = tsb.abi.tsb_plan_stage_times(plan.handle)[dom]
    dom_launch_ms = dom_ms / dom_calls
    log(f"timed region: {dom} mean {dom_launch_ms:.4f} ms per launch over {dom_calls} launches")
    dur_s = dom_launch_ms * 1e-3
    achieved = bytes_alg[dom] / dur_s / 1e9
    traffic = load_traffic(args.workload, plan_geometry(info, req), dom)
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "bytes_per_launch": int(bytes_alg[dom]), "mean_launch_ms": round(dom_launch_ms, 4)}
    if dom == "reduce":
        # the reduction is a contraction on the matrix cores fed by FFT and
        # Q-row work; its FP32 operations per launch (plan info) over the same
        # mean time against the FP32 peak are the primary figure, its HBM rate
        # is kept beside them
        tfl = info.reduce_flops / dur_s / 1e12
        roof.update({"bound": "mfma", "achieved": round(tfl, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tfl / FP32_PEAK_TFLOPS, 4), "flops_per_launch": int(info.reduce_flops),
                     "hbm_achieved_gbs": round(achieved, 1), "hbm_peak_gbs": HBM_PEAK_GBS,
                     "hbm_frac": round(achieved / HBM_PEAK_GBS, 4)})
    mult = "+".join("B_" + "".join(map(str, m)) for m in req["multipoles"])
    if args.workload == "box256" and args.pairs == "diagonal":
        metric = "mocks/sec for B_000+B_202 diagonal k-bin pairs (k1 = k2) at 256^3"
        desc = ("256^3 box, L=1000 Mpc/h, TSC+interlacing, local LOS from an observer 1500 Mpc/h "
                "below the centre, 20 shells dk=0.01 h/Mpc, B_000 + B_202 on the 20 diagonal pairs, "
                "seeded lognormal+Kaiser mocks, N_p log-uniform in [3e5, 3e6]")
    elif args.workload == "box256":
        metric = "mocks/sec for B_000+B_202 all k-bin pairs at 256^3"
        desc = ("256^3 box, L=1000 Mpc/h, TSC+interlacing, local LOS from an observer 1500 Mpc/h "
                "below the centre, 20 shells dk=0.01 h/Mpc, B_000 (210 pairs) + B_202 (400 pairs), "
                "seeded lognormal+Kaiser mocks, N_p log-uniform in [3e5, 3e6]")
    elif args.workload == "box128":
        metric = f"mocks/sec for {mult} all k-bin pairs at 128^3"
        desc = ("128^3 box, L=1000 Mpc/h, 500k particles, TSC+interlacing, local LOS from an observer 1500 Mpc/h "
                "below the centre, 20 shells dk=0.01 h/Mpc, seeded lognormal+Kaiser mock")
    else:
        metric = f"mocks/sec for {mult} all k-bin pairs, 256^3 survey window"
        desc = ("256^3 grid, L=2000 Mpc/h, 2M galaxies in the half shell 500-1000 Mpc/h about the observer, "
                "20M randoms, FKP P0=1e4, TSC+interlacing, 25 shells dk=0.008 h/Mpc, seeded lognormal+Kaiser mock")
    if args.vertex != "x3":
        which = "first" if args.vertex == "x1" else "second"
        metric += f", LOS at the {which} vertex"
        desc += f"; LOS at the {which} vertex (App. B)"
    out = {
        "metric": metric,
        "value": round(value, 3), "unit": "mocks/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc,
                   "seeds": seeds, "n_particles_mean": int(n_mean), "reduction_grid": info.m,
                   "fused_reduction": bool(fused), "autotune": tune},
        "roofline": roof,
        "stage_ms": {k: round(v, 4) for k, v in per_launch.items()},
    }
    plan.close()
    if not args.no_batch and args.workload == "box256" and args.pairs == "paper" and args.vertex == "x3":
        log("concurrent leg ...")
        out["concurrent"] = concurrent_leg(tsb, torch, devs, autotune=not args.no_autotune)
        log(f"concurrent: {out['concurrent']}")
    if not args.no_batch:
        pool = _pool(tsb, [(n, seeds) for n, seeds in BATCH_CLASSES], args.pool)
        log("batched leg ...")
        out["batched"] = batch_leg(tsb, torch, pool, args.pool, args.batch_replicas, not args.no_autotune)
        log(f"batched: {out['batched']}")
        del pool
    if not args.no_serve:
        log("serving leg ...")
        big = serve_catalogue(tsb)
        out["serving"] = serve_leg(tsb, torch, big, args.serve_requests, args.serve_rate, args.serve_slots,
                                   args.serve_budget_gb)
        log(f"serving: {out['serving']}")
        del big
    if not args.no_cpu_baseline and args.workload in ("box256", "box128"):
        log("timing the oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(cats[0], req)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
