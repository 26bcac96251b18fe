#!/usr/bin/env python3
"""Benchmark: DD(r) autocorrelation of N = 10^6 clustered points in a periodic
L = 420 box, 20 log bins in [0.1, 25], on one MI355X.

One step is one full counting call on device-resident inputs: gridding, work
list, pair sweep, binary64 recheck, finalize and the copy of the bins to the
host.  The headline metric is W_ref / t_step in Gpair-evals/s, where W_ref is
the number of unordered candidate pairs of the paper's default cell grid
(cubic cells one reach wide, 27 neighbours, unique pairs only) -- a fixed,
grid-independent measure of the work, so runs with different internal grids
or precisions are comparable.

Prints one JSON line (see --help).  With --gpus N > 1 it exits: the
benchmark measures a single GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

L_BOX = 420.0
N_POINTS = 1_000_000
EDGES = synth.log_edges(0.1, 25.0, 20)
SEED = 2
FLOPS_PER_PAIR = 8          # 3 subtractions, 1 multiply, 2 fused multiply-adds
# MI355X's published float32 vector peak (packed FMA: 256 CU x 64 lanes x 2
# pairs x 2 FLOP x 2.4 GHz); the kernels are built without packed float32
# instructions, so their issue ceiling is half of it
PEAK_FP32 = 157.3           # TFLOP/s
ISSUE_CEILING_FP32 = 78.6   # TFLOP/s, one 64-lane FMA per SIMD per 4 cycles
HBM_PEAK_GBPS = 8000.0
# gridding: 48 bytes read and 40 written per point (input coordinates and
# records in; sorted float32 and binary64 copies, cell ids out), the
# algorithmic traffic of a counting sort of the points by cell
GRID_BYTES_PER_POINT = 88
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_r_fp32_n1e6_traffic.txt")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "sweep_r_fp32_n1e6_counters.txt")
SWEEP_SRC = os.path.join(ROOT, "paper_1911_03545_amd", "csrc", "pc_sweep.hip")


def workload():
    pts = synth.clustered_box(N_POINTS, L_BOX, seed=SEED, nblobs=5000, sigma=2.0)
    return pts


def ref_pairs(pts: np.ndarray, L: float, rmax: float) -> int:
    """Unordered candidate pairs of the paper's default grid: cubic cells of
    side >= rmax (n = floor(L / rmax) reduced until the side exceeds rmax by
    the planner's margin), each cell against itself (n(n-1)/2) and its 13
    forward neighbours with periodic wrap."""
    need = rmax * (1 + 2 ** -28) + L * 2 ** -40
    n = int(np.floor(L / need))
    while n > 1 and L / n < need:
        n -= 1
    idx = np.minimum((pts * (n / L)).astype(np.int64), n - 1)
    cid = (idx[:, 0] * n + idx[:, 1]) * n + idx[:, 2]
    C = np.bincount(cid, minlength=n ** 3).reshape(n, n, n).astype(np.int64)
    total = int((C * (C - 1) // 2).sum())
    offs = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)
            if (dx, dy, dz) > (0, 0, 0)]
    for o in offs:
        total += int((C * np.roll(C, shift=(-o[0], -o[1], -o[2]), axis=(0, 1, 2))).sum())
    return total


def profile_value(path, key):
    """A `key: value` line of a committed rocprofv3 summary, if the summary
    was taken on the current sweep source (else None)."""
    if not os.path.exists(path):
        return None
    src_hash = hashlib.sha256(open(SWEEP_SRC, "rb").read()).hexdigest()[:16]
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("sweep_source_sha256_16") != src_hash:
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def valu_fractions(t_sweep_s: float, candidates: int):
    """The sweep's VALU use three ways, from the committed SQ_INSTS_VALU count
    of the same launch (per dispatch) and the live sweep time: (1) VALU
    lane-operations over the packed float32 lane-operation peak (256 CU x 64
    lanes x 2 x 2.4 GHz = 78.6e12/s), and over the non-packed issue limit
    the kernels are compiled for (half that: packed float32 is disabled); (2) useful-op efficiency, 6 lane-operations
    per candidate pair (3 subtractions, a multiply, 2 fused multiply-adds) over
    the lane-operations executed; (3) their product."""
    insts = profile_value(COUNTERS_FILE, "valu_insts_per_dispatch")
    if insts is None or t_sweep_s <= 0:
        return None
    lane_ops = insts * 64.0
    util = lane_ops / (t_sweep_s * 78.6e12)
    useful = 6.0 * candidates / lane_ops
    return {"valu_lane_ops_per_launch": lane_ops,
            "utilisation_vs_packed_peak": util,
            "utilisation_vs_issue_limit": 2.0 * util,
            "useful_op_efficiency": useful,
            "algorithmic_fraction": util * useful}


def gridding_fraction(t_grid_ms: float, n_points: int):
    """Gridding (cell index, counting sort, sorted copies) as a fraction of
    the HBM peak: GRID_BYTES_PER_POINT x points over its measured time."""
    if not t_grid_ms or t_grid_ms <= 0:
        return None
    gbps = GRID_BYTES_PER_POINT * n_points / (t_grid_ms / 1e3) / 1e9
    return {"ms": t_grid_ms, "bytes_per_point": GRID_BYTES_PER_POINT,
            "achieved_GBps": gbps, "peak_GBps": HBM_PEAK_GBPS,
            "frac": gbps / HBM_PEAK_GBPS}


def read_traffic():
    """HBM bytes per sweep launch from the committed rocprofv3 counter
    summary, if it was taken on the current sweep source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    src_hash = hashlib.sha256(open(SWEEP_SRC, "rb").read()).hexdigest()[:16]
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("sweep_source_sha256_16") != src_hash:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(pts: np.ndarray, w_ref: int, target_s: float = 12.0):
    """The CPU oracle, untuned, on a bounded sample of the same workload:
    cross-counts of a random subset S against all N points.  Its brute-force
    pair rate is scaled to the full workload (N(N-1)/2 unique pairs) and
    expressed in the metric's unit, W_ref / t_full."""
    import oracle
    lib = oracle.load()
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    rng = synth.rng_for(99)
    # calibrate on growing samples until one takes a measurable time, then
    # size the sample to ~target_s
    m0 = 64
    while True:
        s0 = pts[rng.choice(pts.shape[0], m0, replace=False)]
        t = time.perf_counter()
        oracle.count_r(s0, pts, EDGES, L_BOX, nthreads=cores, lib=lib)
        dt = time.perf_counter() - t
        if dt > 0.5 or m0 >= pts.shape[0]:
            break
        m0 = min(pts.shape[0], m0 * 4)
    # three samples of a third of the target each; the median rate counts
    m = int(min(pts.shape[0], max(64, m0 * target_s / 3.0 / dt)))
    rates, els = [], []
    for _ in range(3):
        sample = pts[rng.choice(pts.shape[0], m, replace=False)]
        t = time.perf_counter()
        oracle.count_r(sample, pts, EDGES, L_BOX, nthreads=cores, lib=lib)
        els.append(time.perf_counter() - t)
        rates.append(m * pts.shape[0] / els[-1])
    k = int(np.argsort(rates)[1])
    rate, el = rates[k], els[k]                  # brute-force pair evaluations / s
    full_pairs = pts.shape[0] * (pts.shape[0] - 1) / 2
    t_full = full_pairs / rate
    # one thread on a sample of about 3 s, for the per-core rate
    m1 = max(16, int(m * 3.0 / max(el, 1e-9) / cores))
    s1 = pts[rng.choice(pts.shape[0], min(m1, pts.shape[0]), replace=False)]
    t = time.perf_counter()
    oracle.count_r(s1, pts, EDGES, L_BOX, nthreads=1, lib=lib)
    el1 = time.perf_counter() - t
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": w_ref / t_full / 1e9,
        "unit": "Gpair-evals/s",
        "cores": cores,
        "kind": "oracle",
        "nproc": os.cpu_count(),
        "cpu_model": model,
        "single_thread_gpair_per_s": s1.shape[0] * pts.shape[0] / el1 / 1e9,
        "sample": (f"brute-force cross counts of {m} random points against all "
                   f"{pts.shape[0]}, three samples, the median: {m * pts.shape[0]:.3g} pair "
                   f"evaluations in {el:.1f} s, {rate / 1e9:.3f} Gpair/s; full auto workload "
                   f"of {full_pairs:.3g} unique pairs extrapolated to {t_full:.0f} s"),
    }


def batch_bench(args, steps=None, emit=True):
    """Batched DD(rp, pi): 256 (--batch-cats) clustered mock catalogues of 2e5-2e6 points in
    periodic L = 1000 boxes, 20 log rp bins in [0.1, 25], pimax = 40 in 40
    bins.  Reports the 2x2 ablation {binary64, float32 + recheck} x {256
    sequential calls, one batched call replayed from a graph}, as Gpair-evals/s
    over the sum of the catalogues' reference candidate pairs.  Returns the
    result line (printed when `emit`)."""
    import torch
    import paper_1911_03545_amd as pcm

    steps = args.steps if steps is None else steps

    dev = torch.device("cuda:0")
    L = 1000.0
    sizes = synth.batch_sizes(args.batch_cats, 200_000, 2_000_000, seed=5)
    edges = synth.log_edges(0.1, 25.0, 20)
    cats, w_ref = [], 0
    t = time.perf_counter()
    for c, n in enumerate(sizes):
        pts = synth.clustered_box(int(n), L, seed=5000 + c, nblobs=max(1, int(n) // 200),
                                  sigma=2.0)
        w_ref += ref_pairs_rppi(pts, L, 25.0, 40.0)
        cats.append(tuple(torch.from_numpy(np.ascontiguousarray(pts[:, k])).to(dev)
                          for k in range(3)))
        if (c + 1) % 32 == 0:
            print(f"generated {c + 1}/{len(sizes)} catalogues", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t
    ctx = pcm.PairCounter(0, stream=torch.cuda.current_stream(dev))

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps, out

    res = {}
    ref = None
    for prec in ("fp32", "fp64"):
        opts = pcm.default_options(use_graph=1, autotune=1)
        tb, (cb, _) = timed(lambda: ctx.count_rppi_batch(cats, edges, 40.0, 40, L, prec,
                                                         options=opts), steps)
        st = ctx.stats()
        print(f"{prec}: batched {tb * 1e3:.2f} ms", file=sys.stderr, flush=True)
        sopts = pcm.default_options(autotune=1)

        def seq():
            return np.stack([ctx.count_rppi(cc, None, edges, 40.0, 40, L, prec,
                                            options=sopts)[0] for cc in cats])
        if args.batch_only:
            ts, cs = float("nan"), cb
        else:
            ts, cs = timed(seq, max(1, steps // 5))
        print(f"{prec}: sequential {ts * 1e3:.2f} ms", file=sys.stderr, flush=True)
        if ref is None:
            ref = cb
        if not (np.array_equal(cb, ref) and np.array_equal(cs, ref)):
            raise SystemExit("batched and sequential counts differ")
        res[prec] = {"batched_graph_ms": tb * 1e3, "sequential_ms": ts * 1e3,
                     "batched_value": w_ref / tb / 1e9, "sequential_value": w_ref / ts / 1e9,
                     "candidate_pairs": st["candidate_pairs"], "rechecks": st["rechecks"],
                     "slices_per_reach": st["slices_per_reach"], "chunk": st["chunk"],
                     "xy_refine": st["xy_refine"],
                     "replayed": st["replayed"]}
    line = {
        "metric": f"Gpair-evals/s for batched DD(rp,pi), {len(sizes)} mocks, FP32+recheck "
                  "batched vs plain FP64 sequential",
        "value": res["fp32"]["batched_value"],
        "unit": "Gpair-evals/s",
        "n_gpus": 1,
        "steps": steps,
        "higher_is_better": True,
        "vs_plain_fp64_sequential": res["fp32"]["batched_value"] / res["fp64"]["sequential_value"],
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(sizes)} clustered catalogues (N_c/200 blobs, sigma 2) of "
                               f"{int(sizes.min())}-{int(sizes.max())} points, periodic L=1000, "
                               "20 log rp bins [0.1, 25], pimax 40 / 40 bins, float64 inputs",
                   "total_points": int(sizes.sum()), "w_ref_pairs": int(w_ref),
                   "generation_s": gen_s},
        "ablation": res,
    }
    ctx.close()
    del cats
    torch.cuda.empty_cache()
    if emit:
        print(json.dumps(line), flush=True)
    return line


def ref_pairs_box(v: np.ndarray, reach: float) -> int:
    """Unordered candidate pairs of the paper's default grid for a
    non-periodic catalogue: cubic cells of side >= reach over the bounding
    box, each cell against itself and its 13 forward neighbours."""
    lo, hi = v.min(axis=0), v.max(axis=0)
    ext = np.maximum(hi - lo, reach)
    n = np.maximum(np.floor(ext / (reach * (1 + 2 ** -28))).astype(np.int64), 1)
    idx = [np.minimum(((v[:, a] - lo[a]) * (n[a] / ext[a])).astype(np.int64), n[a] - 1)
           for a in range(3)]
    cid = (idx[0] * n[1] + idx[1]) * n[2] + idx[2]
    C = np.bincount(cid, minlength=int(n.prod())).reshape(n).astype(np.int64)
    total = int((C * (C - 1) // 2).sum())
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                if (dx, dy, dz) <= (0, 0, 0):
                    continue
                a = C[max(0, -dx):n[0] - max(0, dx), max(0, -dy):n[1] - max(0, dy),
                      max(0, -dz):n[2] - max(0, dz)]
                b = C[max(0, dx):n[0] - max(0, -dx) if dx < 0 else n[0],
                      max(0, dy):n[1] - max(0, -dy) if dy < 0 else n[1],
                      max(0, dz):n[2] - max(0, -dz) if dz < 0 else n[2]]
                total += int((a * b).sum())
    return total


def mocks_bench(args):
    """On-sky DD(rp, pi) (line of sight through each pair's midpoint) of a
    clustered 10^6-point mock: a 10-degree cone between distances 500 and
    1500, half the points in 3-D Gaussian blobs (100 points, width 2); 20
    log rp bins [0.1, 25], pimax 40 in 40 bins; RA/DEC/distance converted on
    the device.  The value is pair evaluations per second (the sweep's
    candidate pairs per step over the step time), and, for scale, the same
    for the untuned oracle on a bounded sample."""
    import torch
    import paper_1911_03545_amd as pcm
    t0 = time.perf_counter()
    m = synth.sky_mock(1_000_000, seed=2024)
    gen_s = time.perf_counter() - t0
    e = synth.log_edges(0.1, 25.0, 20)
    dev = torch.device("cuda:0")
    cols = tuple(torch.from_numpy(np.ascontiguousarray(m[:, k])).to(dev) for k in range(3))
    torch.cuda.synchronize()
    import oracle
    lib = oracle.load()
    v = oracle.sky_to_cartesian(m[:, 0], m[:, 1], m[:, 2], lib=lib)
    w_ref = ref_pairs_box(v, float(np.sqrt(25.0 ** 2 + 40.0 ** 2)))
    ctx = pcm.PairCounter(0, stream=torch.cuda.current_stream(dev))
    opts = pcm.default_options(collect_timing=1)
    for _ in range(args.warmup):
        counts, _ = ctx.count_rppi_mocks(cols, None, e, 40.0, 40, "fp64", options=opts)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        counts, _ = ctx.count_rppi_mocks(cols, None, e, 40.0, 40, "fp64", options=opts)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / args.steps
    st = ctx.stats()
    cand = st["candidate_pairs"]
    line = {
        "metric": "Gpair-evals/s for on-sky DD(rp,pi) N=1e6 (binary64; reference pairs of "
                  "the paper's cells of side sqrt(rpmax^2 + pimax^2))",
        "value": w_ref / (ms / 1e3) / 1e9,
        "unit": "Gpair-evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "on-sky DD(rp,pi) autocorrelation, 1e6 clustered points in a "
                               "10-degree cone, distances 500-1500, 20 log rp bins [0.1, 25], "
                               "pimax 40 / 40 bins, RA/DEC/distance float64 inputs in HBM",
                   "w_ref_pairs": w_ref, "generation_s": gen_s},
        "sweep": {"kernel_ms": st["t_sweep_ms"], "candidate_pairs": cand,
                  "candidate_over_ref": cand / w_ref,
                  "in_range_pairs": int(counts.sum()), "grid": st["grid"],
                  "phase_ms": {k: st[k] for k in ("t_prepare_ms", "t_grid_ms",
                                                  "t_worklist_ms", "t_sweep_ms",
                                                  "t_finalize_ms", "t_total_ms")}},
    }
    if not args.no_cpu_baseline:
        cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
        rng = synth.rng_for(98)
        # calibrate on growing samples, then size the sample to ~12 s
        k = 256
        while True:
            sample = v[rng.choice(v.shape[0], k, replace=False)]
            t = time.perf_counter()
            oracle.count_rppi_mocks(sample, v, e, 40.0, 40, nthreads=cores, lib=lib)
            el = time.perf_counter() - t
            if el > 0.5 or k >= v.shape[0]:
                break
            k = min(v.shape[0], k * 4)
        k = int(min(v.shape[0], max(256, k * 12.0 / el)))
        sample = v[rng.choice(v.shape[0], k, replace=False)]
        t = time.perf_counter()
        oracle.count_rppi_mocks(sample, v, e, 40.0, 40, nthreads=cores, lib=lib)
        el = time.perf_counter() - t
        rate = k * v.shape[0] / el
        t_full = v.shape[0] * (v.shape[0] - 1) / 2 / rate
        line["cpu_baseline"] = {
            "value": w_ref / t_full / 1e9, "unit": "Gpair-evals/s", "cores": cores,
            "kind": "oracle",
            "sample": f"brute-force cross counts of {k} random points against all "
                      f"{v.shape[0]} ({k * v.shape[0]:.3g} pair evaluations in {el:.1f} s, "
                      f"{rate / 1e9:.3f} Gpair/s); full auto workload extrapolated to "
                      f"{t_full:.0f} s"}
    ctx.close()
    print(json.dumps(line), flush=True)


def ref_pairs_box_cross(v1: np.ndarray, v2: np.ndarray, reach: float) -> int:
    """Cross-correlation candidate pairs of the paper's default grid: cubic
    cells of side >= reach over the joint bounding box, each cell of the
    first catalogue against the 27 cells around it in the second."""
    lo = np.minimum(v1.min(axis=0), v2.min(axis=0))
    hi = np.maximum(v1.max(axis=0), v2.max(axis=0))
    ext = np.maximum(hi - lo, reach)
    n = np.maximum(np.floor(ext / (reach * (1 + 2 ** -28))).astype(np.int64), 1)

    def hist(v):
        idx = [np.minimum(((v[:, a] - lo[a]) * (n[a] / ext[a])).astype(np.int64), n[a] - 1)
               for a in range(3)]
        cid = (idx[0] * n[1] + idx[1]) * n[2] + idx[2]
        return np.bincount(cid, minlength=int(n.prod())).reshape(n).astype(np.int64)

    A, B = hist(v1), hist(v2)
    Bp = np.pad(B, 1)
    total = 0
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                total += int((A * Bp[1 + dx:1 + dx + n[0], 1 + dy:1 + dy + n[1],
                                     1 + dz:1 + dz + n[2]]).sum())
    return total


def theta_bench(args):
    """DD(theta) and DR(theta) on a 30-degree cap centred at (RA, DEC) =
    (0, 30) (across the RA seam): D = 2e6 points, half uniform, half in
    10 000 Gaussian blobs of width 0.1 degree; R = 5e6 uniform; 20 log bins in
    [0.01, 10] degrees; RA/DEC float64 in HBM.  Each statistic runs on the 3-D
    chord grid and on the angular grid (declination bands, right-ascension
    cells 1/n of the reach, n = 4, 8 (the default), 16; 32 declination slices
    per band), in float32 + recheck and binary64.
    Values are reference pairs (the paper's cubic cells of side
    2 sin(5 degrees) on the unit vectors) per second."""
    import torch
    import paper_1911_03545_amd as pcm
    import oracle
    t0 = time.perf_counter()
    ra, dec = synth.cap_radec(2_000_000, seed=4, radius_deg=30.0, clustered=True)
    rr, rd = synth.cap_radec(5_000_000, seed=40, radius_deg=30.0)
    gen_s = time.perf_counter() - t0
    te = synth.log_edges(0.01, 10.0, 20)
    lib = oracle.load()
    vd = oracle.radec_to_unit(ra, dec, lib=lib)
    vr = oracle.radec_to_unit(rr, rd, lib=lib)
    reach = 2.0 * np.sin(0.5 * np.deg2rad(10.0))
    wref = {"DD": ref_pairs_box(vd, reach), "DR": ref_pairs_box_cross(vd, vr, reach)}
    dev = torch.device("cuda:0")
    D = tuple(torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (ra, dec))
    R = tuple(torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (rr, rd))
    torch.cuda.synchronize()
    ctx = pcm.PairCounter(0, stream=torch.cuda.current_stream(dev))
    runs = {}
    ref_counts = {}
    for stat in ("DD", "DR"):
        other = (None, None) if stat == "DD" else R
        for prec in args.theta_precisions.split(","):
            for grid in (int(g) for g in args.theta_grids.split(",")):
                opts = pcm.default_options(collect_timing=1, angular_grid=grid)

                def call():
                    return ctx.count_theta(D[0], D[1], other[0], other[1], te, prec,
                                           options=opts)
                for _ in range(args.warmup):
                    counts, _ = call()
                torch.cuda.synchronize()
                t = time.perf_counter()
                for _ in range(args.steps):
                    counts, _ = call()
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t) * 1e3 / args.steps
                st = ctx.stats()
                if stat not in ref_counts:
                    ref_counts[stat] = counts.copy()
                elif not np.array_equal(ref_counts[stat], counts):
                    raise SystemExit(f"{stat} counts differ between grids / precisions")
                key = f"{stat}_{prec}_" + ("chord" if grid < 0 else f"angular{grid}")
                runs[key] = {"ms_per_step": ms,
                             "value": wref[stat] / (ms / 1e3) / 1e9,
                             "sweep_ms": st["t_sweep_ms"],
                             "candidate_pairs": st["candidate_pairs"],
                             "candidate_over_ref": st["candidate_pairs"] / wref[stat],
                             "grid": st["grid"]}
                print(key, json.dumps(runs[key]), flush=True)
    dd = [k for k in runs if k.startswith("DD_")]
    best = min((k for k in dd if "_fp32_" in k) or dd, key=lambda k: runs[k]["ms_per_step"])
    line = {
        "metric": "Gpair-evals/s for DD(theta) N=2e6 on a 30-degree cap (reference pairs of "
                  "the paper's cubic cells on the unit vectors)",
        "value": runs[best]["value"], "unit": "Gpair-evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": runs[best]["ms_per_step"], "higher_is_better": True,
        "dtype": "f32" if "_fp32_" in best else "f64",
        "data": "synthetic",
        "config": {"workload": "DD(theta) / DR(theta): D 2e6 (half in 10000 blobs of 0.1 deg), "
                               "R 5e6 uniform, 30-degree cap at (0, 30) across the RA seam, "
                               "20 log bins [0.01, 10] deg, RA/DEC float64 in HBM",
                   "best": best, "w_ref_pairs": wref, "generation_s": gen_s},
        "runs": runs,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


def weighted_bench(args):
    """Weighted counts of 4e6 clustered points (20000 Gaussian blobs of width
    2 holding half of them) in a periodic L = 1100 box with float32 weights
    uniform in [0.5, 1.5) and product pair weights: xi(r) counts with 25 log
    bins in [0.1, 50], and wp(rp) counts with the same rp bins, pimax 40 in 40
    bins; each in float32 + recheck and in binary64, with binary64 atomic
    weight sums and with exact fixed-point sums (deterministic_weights).
    Reports time per call, reference pairs per second, and the weighted sums'
    agreement: float32 + recheck against binary64 over the whole catalogue,
    and against the oracle on sampled cross counts (256 points against all);
    the fixed-point sums must equal across precisions and equal the oracle's
    exactly rounded sums bit for bit."""
    import torch
    import paper_1911_03545_amd as pcm
    import oracle
    L = 1100.0
    t0 = time.perf_counter()
    pts = synth.clustered_box(4_000_000, L, seed=3, nblobs=20000, sigma=2.0)
    w = synth.uniform_weights(4_000_000, seed=33)
    gen_s = time.perf_counter() - t0
    e = synth.log_edges(0.1, 50.0, 25)
    wref = {"r": ref_pairs(pts, L, 50.0), "rppi": ref_pairs_rppi(pts, L, 50.0, 40.0)}
    dev = torch.device("cuda:0")
    cols = tuple(torch.from_numpy(np.ascontiguousarray(pts[:, k])).to(dev) for k in range(3))
    wd = torch.from_numpy(w).to(dev)
    torch.cuda.synchronize()
    ctx = pcm.PairCounter(0, stream=torch.cuda.current_stream(dev))
    opts = pcm.default_options(collect_timing=1)
    lib = oracle.load()
    idx = np.sort(synth.rng_for(77).choice(pts.shape[0], size=256, replace=False))
    runs = {}
    for stat in ("r", "rppi"):
        sums = {}
        for prec in ("fp32", "fp64"):
            if stat == "r":
                def call():
                    return ctx.count_r(cols, None, e, L, prec, w1=wd, options=opts)
            else:
                def call():
                    return ctx.count_rppi(cols, None, e, 40.0, 40, L, prec, w1=wd, options=opts)
            for _ in range(args.warmup):
                c, ws = call()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.steps):
                c, ws = call()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t) * 1e3 / args.steps
            st = ctx.stats()
            sums[prec] = (c, ws)
            runs[f"{stat}_{prec}"] = {"ms_per_step": ms, "value": wref[stat] / (ms / 1e3) / 1e9,
                                      "sweep_ms": st["t_sweep_ms"],
                                      "candidate_pairs": st["candidate_pairs"],
                                      "rechecks": st["rechecks"]}
        if not np.array_equal(sums["fp32"][0], sums["fp64"][0]):
            raise SystemExit(f"{stat}: float32 + recheck and binary64 counts differ")
        fixed = {}
        fopts = pcm.default_options(collect_timing=1, deterministic_weights=1)
        for prec in ("fp32", "fp64"):
            if stat == "r":
                def call():
                    return ctx.count_r(cols, None, e, L, prec, w1=wd, options=fopts)
            else:
                def call():
                    return ctx.count_rppi(cols, None, e, 40.0, 40, L, prec, w1=wd,
                                          options=fopts)
            for _ in range(args.warmup):
                c, ws = call()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.steps):
                c, ws = call()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t) * 1e3 / args.steps
            fixed[prec] = ws
            runs[f"{stat}_{prec}_fixed_sums"] = {
                "ms_per_step": ms, "value": wref[stat] / (ms / 1e3) / 1e9,
                "sweep_ms": ctx.stats()["t_sweep_ms"]}
        if not np.array_equal(fixed["fp32"], fixed["fp64"]):
            raise SystemExit(f"{stat}: fixed-point weight sums differ between precisions")
        a, b = sums["fp32"][1], sums["fp64"][1]
        nz = b != 0
        runs[f"{stat}_wsum_rel_fp32_vs_fp64"] = float(np.max(np.abs(a[nz] - b[nz]) / np.abs(b[nz])))
        # sampled cross counts against the oracle's exactly rounded sums
        if stat == "r":
            g, gw = ctx.count_r(pts[idx], pts, e, L, "fp32", w1=w[idx], w2=w)
            o, ow = oracle.count_r(pts[idx], pts, e, L, w1=w[idx], w2=w, lib=lib)
        else:
            g, gw = ctx.count_rppi(pts[idx], pts, e, 40.0, 40, L, "fp32", w1=w[idx], w2=w)
            o, ow = oracle.count_rppi(pts[idx], pts, e, 40.0, 40, L, w1=w[idx], w2=w, lib=lib)
        if not np.array_equal(g, o):
            raise SystemExit(f"{stat}: sampled counts differ from the oracle")
        nz = ow != 0
        runs[f"{stat}_wsum_rel_vs_oracle_sampled"] = float(
            np.max(np.abs(gw[nz] - ow[nz]) / np.abs(ow[nz])))
        det = {"deterministic_weights": 1}
        if stat == "r":
            _, fw = ctx.count_r(pts[idx], pts, e, L, "fp32", w1=w[idx], w2=w, options=det)
        else:
            _, fw = ctx.count_rppi(pts[idx], pts, e, 40.0, 40, L, "fp32", w1=w[idx], w2=w,
                                   options=det)
        if not np.array_equal(fw, ow):
            raise SystemExit(f"{stat}: fixed-point sums differ from the oracle's")
        runs[f"{stat}_fixed_sums_equal_oracle_sampled"] = True
    line = {
        "metric": "Gpair-evals/s for weighted xi(r) / wp(rp) counts, N=4e6 periodic L=1100 "
                  "(reference pairs of the paper's cells)",
        "value": runs["r_fp32"]["value"], "unit": "Gpair-evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": runs["r_fp32"]["ms_per_step"], "higher_is_better": True, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "weighted DD(r) and DD(rp,pi), 4e6 clustered points (half in "
                               "20000 blobs, sigma 2), periodic L=1100, float32 weights "
                               "U[0.5,1.5), product pair weights, 25 log bins [0.1, 50], "
                               "pimax 40 / 40 bins, float64 inputs in HBM",
                   "w_ref_pairs": wref, "generation_s": gen_s},
        "runs": runs,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


def ref_pairs_rppi(pts: np.ndarray, L: float, rpmax: float, pimax: float) -> int:
    """Unordered candidate pairs of the paper's default grid for rp/pi: cells
    of side >= rpmax in x, y and >= pimax along z, 13 forward neighbours plus
    the pairs inside each cell."""
    n = []
    for reach in (rpmax, rpmax, pimax):
        need = reach * (1 + 2 ** -28) + L * 2 ** -40
        k = int(np.floor(L / need))
        while k > 1 and L / k < need:
            k -= 1
        n.append(k)
    idx = [np.minimum((pts[:, a] * (n[a] / L)).astype(np.int64), n[a] - 1) for a in range(3)]
    cid = (idx[0] * n[1] + idx[1]) * n[2] + idx[2]
    C = np.bincount(cid, minlength=n[0] * n[1] * n[2]).reshape(n).astype(np.int64)
    total = int((C * (C - 1) // 2).sum())
    offs = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)
            if (dx, dy, dz) > (0, 0, 0)]
    for o in offs:
        total += int((C * np.roll(C, shift=(-o[0], -o[1], -o[2]), axis=(0, 1, 2))).sum())
    return total


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain-FP64 comparison run")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the graph-replay and mean-separation runs (profiling)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy a MIB-sized device buffer three times (a kernel of "
                         "known traffic for scaling hardware byte counters)")
    ap.add_argument("--batch", action="store_true",
                    help="run the batched DD(rp,pi) benchmark (256 mock catalogues) instead")
    ap.add_argument("--batch-cats", type=int, default=256)
    ap.add_argument("--no-batch", action="store_true",
                    help="leave the batched 256-catalogue ablation out of the default line")
    ap.add_argument("--batch-steps", type=int, default=3,
                    help="timed batched calls per precision in the default line's ablation")
    ap.add_argument("--batch-only", action="store_true",
                    help="with --batch: time only the batched calls (no sequential cells; "
                         "for profiling)")
    ap.add_argument("--mocks", action="store_true",
                    help="run the on-sky DD(rp,pi) benchmark (1e6-point mock) instead")
    ap.add_argument("--theta", action="store_true",
                    help="run the DD(theta)/DR(theta) benchmark (2e6 + 5e6 points on a cap, "
                         "chord and angular grids) instead")
    ap.add_argument("--weighted", action="store_true",
                    help="run the weighted xi(r) / wp(rp) benchmark (4e6 points, L=1100) instead")
    ap.add_argument("--theta-grids", default="-1,8,16,32",
                    help="angular_grid values for --theta (-1: 3-D chord grid)")
    ap.add_argument("--theta-precisions", default="fp32,fp64")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures the single-GPU path only; "
                                   "--gpus must be 1 (how the path would shard over "
                                   "several GPUs is a design note, not a measured mode)"}))
        sys.exit(2)

    if args.batch:
        batch_bench(args)
        return
    if args.mocks:
        mocks_bench(args)
        return
    if args.theta:
        theta_bench(args)
        return
    if args.weighted:
        weighted_bench(args)
        return
    import torch
    import paper_1911_03545_amd as pcm

    dev = torch.device("cuda:0")
    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * (1 << 18), dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    pts = workload()
    w_ref = ref_pairs(pts, L_BOX, EDGES[-1])
    cols = tuple(torch.from_numpy(np.ascontiguousarray(pts[:, k])).to(dev) for k in range(3))
    torch.cuda.synchronize()
    ctx = pcm.PairCounter(0, stream=torch.cuda.current_stream(dev))
    opts = pcm.default_options(collect_timing=1)

    def run(prec):
        return ctx.count_r(cols, None, EDGES, L_BOX, prec, options=opts)

    for _ in range(args.warmup):
        counts, _ = run(args.precision)
    torch.cuda.synchronize()
    sweep_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        counts, _ = run(args.precision)
        sweep_ms.append(ctx.stats()["t_sweep_ms"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = ctx.stats()
    ms = elapsed * 1e3 / args.steps
    value = w_ref / (ms / 1e3) / 1e9

    fp64 = None
    if not args.no_fp64 and args.precision == "fp32":
        c64, _ = run("fp64")
        for _ in range(2):
            run("fp64")
        torch.cuda.synchronize()
        t = time.perf_counter()
        k64 = max(5, args.steps // 5)
        for _ in range(k64):
            run("fp64")
        torch.cuda.synchronize()
        ms64 = (time.perf_counter() - t) * 1e3 / k64
        if not np.array_equal(c64, counts):
            raise SystemExit("fp32+recheck and fp64 counts differ")
        fp64 = {"value": w_ref / (ms64 / 1e3) / 1e9, "ms_per_step": ms64,
                "sweep_ms": ctx.stats()["t_sweep_ms"]}

    # the same call replayed from a recorded HIP graph (repeated identical
    # calls on the same device buffers; every kernel still runs)
    graph = None
    if not args.no_extras:
        gopts = pcm.default_options(use_graph=1)
        cg, _ = ctx.count_r(cols, None, EDGES, L_BOX, args.precision, options=gopts)
        for _ in range(3):
            ctx.count_r(cols, None, EDGES, L_BOX, args.precision, options=gopts)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            cg, _ = ctx.count_r(cols, None, EDGES, L_BOX, args.precision, options=gopts)
        torch.cuda.synchronize()
        msg = (time.perf_counter() - t) * 1e3 / args.steps
        if not np.array_equal(cg, counts):
            raise SystemExit("graph replay and eager counts differ")
        graph = {"ms_per_step": msg, "value": w_ref / (msg / 1e3) / 1e9,
                 "replayed": ctx.stats()["replayed"]}

    # the same call on host-resident columns: each call copies the 24 MB of
    # float64 coordinates over PCIe first (reported, never the headline)
    host = None
    if not args.no_extras:
        hcols = tuple(np.ascontiguousarray(pts[:, k]) for k in range(3))
        ch, _ = ctx.count_r(hcols, None, EDGES, L_BOX, args.precision)
        torch.cuda.synchronize()
        t = time.perf_counter()
        k_host = max(5, args.steps // 5)
        for _ in range(k_host):
            ch, _ = ctx.count_r(hcols, None, EDGES, L_BOX, args.precision)
        torch.cuda.synchronize()
        msh = (time.perf_counter() - t) * 1e3 / k_host
        if not np.array_equal(ch, counts):
            raise SystemExit("host-input and device-input counts differ")
        host = {"ms_per_step": msh, "value": w_ref / (msh / 1e3) / 1e9,
                "input_bytes": int(sum(c.nbytes for c in hcols))}

    # the same workload with the mean separation per bin (one square root
    # and two more LDS sums per pair in range), in both precisions
    ravg = {}
    for prec in (() if args.no_extras else ("fp32", "fp64")):
        cr, _, rv = ctx.count_r(cols, None, EDGES, L_BOX, prec, ravg=True)
        if not np.array_equal(cr, counts):
            raise SystemExit("counts with the mean separation differ")
        torch.cuda.synchronize()
        t = time.perf_counter()
        kr = max(5, args.steps // 5)
        for _ in range(kr):
            ctx.count_r(cols, None, EDGES, L_BOX, prec, options=opts, ravg=True)
        torch.cuda.synchronize()
        msr = (time.perf_counter() - t) * 1e3 / kr
        ravg[prec] = {"value": w_ref / (msr / 1e3) / 1e9, "ms_per_step": msr,
                      "sweep_ms": ctx.stats()["t_sweep_ms"]}

    t_sweep = float(np.mean(sweep_ms)) / 1e3
    achieved = FLOPS_PER_PAIR * st["candidate_pairs"] / t_sweep / 1e12
    line = {
        "metric": "Gpair-evals/s for DD(r) N=1e6 periodic",
        "value": value,
        "unit": "Gpair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "DD(r) autocorrelation, 1e6 clustered points (half uniform, half in "
                        "5000 Gaussian blobs, sigma 2), periodic L=420, 20 log bins "
                        "[0.1, 25], float64 inputs in HBM, "
                        + ("float32 + binary64 recheck" if args.precision == "fp32"
                           else "binary64"),
            "n_points": N_POINTS,
            "boxsize": L_BOX,
            "nbins": 20,
            "w_ref_pairs": w_ref,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32,
            "traffic": read_traffic(),
            "peak_kind": "fp32 vector, packed FMA (published)",
            "issue_ceiling": ISSUE_CEILING_FP32,
            "frac_of_issue_ceiling": achieved / ISSUE_CEILING_FP32,
        },
        "gridding": gridding_fraction(st["t_grid_ms"], N_POINTS),
        "valu": valu_fractions(t_sweep, st["candidate_pairs"]) if args.precision == "fp32"
        else None,
        "sweep": {
            "kernel_ms": t_sweep * 1e3,
            "candidate_pairs": st["candidate_pairs"],
            "candidate_over_ref": st["candidate_pairs"] / w_ref,
            "rechecks": st["rechecks"],
            "grid": st["grid"],
            "zreach": st["zreach"],
            "workgroups": st["sweep_workgroups"],
            "phase_ms": {k: st[k] for k in ("t_prepare_ms", "t_grid_ms", "t_worklist_ms",
                                            "t_sweep_ms", "t_finalize_ms", "t_total_ms")},
        },
        "fp64_path": fp64,
        "graph_replay": graph,
        "host_input_path": host,
        "ravg_path": ravg,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(pts, w_ref)
        # time ratio of the full workload: the oracle's extrapolated time over a GPU call
        line["cpu_baseline"]["gpu_speedup"] = value / line["cpu_baseline"]["value"]
    ctx.close()
    # the metric's second half: the batched workload's 2x2 ablation
    # {binary64, float32 + recheck} x {256 sequential calls, one batched
    # graph-replayed call}, after the timed DD(r) steps
    if not args.no_batch:
        b = batch_bench(args, steps=args.batch_steps, emit=False)
        line["batch_ablation"] = {
            "metric": b["metric"], "unit": b["unit"], "config": b["config"],
            "value_fp32_batched": b["value"],
            "fp32_batched_vs_fp64_sequential": b["vs_plain_fp64_sequential"],
            "cells": b["ablation"], "steps": b["steps"]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
