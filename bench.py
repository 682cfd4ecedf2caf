#!/usr/bin/env python3
"""Benchmark: shifts/s of sigma_min(zI - A) in FP64 on one MI355X.

Workload (the measured configuration): non-normal tridiagonal Toeplitz A, n = 2000
(sub 0.25, diag 0, super 1.0), complex128; 256 x 256 grid on [-2, 2] x [-2, 2].  One step =
the whole hot path over that grid: the full grid through ps_eval_grid (the plain method,
every grid point, with the sensitive-zone epilogue at eps = 1e-2) plus the restricted set of
~25 % of the grid points (an annulus around |z| = 1, seeded) through the mask path of
ps_eval_grid.  The two are independent calls; the mask call runs on a second stream (own
workspace) so that its wavefronts use the SIMDs the full-grid launch frees (--serial: one
stream, back to back).  value = shifts evaluated per second over the timed steps (65536 +
16280 shifts per step), inputs resident in HBM before timing starts.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--serial]
    python bench.py --counter-pass            (under rocprofv3 --pmc: copy calibration + one
                                               full-grid launch, nothing timed)
    python bench.py --summarize-counters FETCH.csv WRITE.csv
                                              (writes profiles/toeplitz2000_traffic.json)

Prints ONE JSON line.  The roofline object prices the dominant kernel (the persistent
eval kernel, full-grid launch).  Most shifts of this workload take the inertia bisection,
whose passes read only the band of A (cached) and keep their state in registers: FP64
arithmetic, so the roofline is "alu" against the FP64 vector peak (78.6 TFLOP/s).  Per row
of a pass, with hb = kl + ku and kt test points per pass (3 for hb <= 2, 2 for hb <= 4,
else 1), counting each FP64 add, multiply and fused multiply-add as executed (an FMA is 2):
  F_row = 4 (hb+1) + 8 hb(hb+1)/2                (H[i][i], real, and H[i][i-e], e = 1..hb)
        + kt (8 hb(hb-1)/2 + 6 hb + 10)         (per test: the factor row of L D L^H, the
                                                 pivot, and 1/pivot: hardware reciprocal
                                                 plus two Newton steps)
and a launch performs F = F_row * n * (sum of the passes of its shifts, from the info word);
every pass covers all n rows.  The shifts on the Golub-Kahan path move
  B_LU   = (w_L + w_U) 16 n + n                 (L, U, pivots written once)
  B_step = (2 (w_L + w_U) + 10) 16 n + 2 n      (factors read twice, ten vector passes,
                                                  pivots read twice) per Lanczos step
plus 16 bytes of output per shift and the band once (w_L = kl, w_U = kl + ku + 1); those
bytes are reported beside the roofline.  Duration: HIP events on the stream the kernel
runs on.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector peak
EPS_ZONE = 1e-2
CALIB_BYTES = 1 << 30          # the calibration copy: 1 GiB read, 1 GiB written
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "toeplitz2000_traffic.json")


# The sources of the measured call: the bisection kernel (half-bandwidth 2) and the
# Golub-Kahan kernel at kl = ku = 1, their workspace carving and launchers, the constants they
# share, and the host side that plans the call.
EVAL_SOURCES = ("ps_bisect.hpp", "ps_bisect.hip", "ps_bis_h2.hip", "ps_eval.hpp", "ps_eval_kl1.hip", "ps_kernels.hip",
                "ps_internal.h", "ps_api.cpp")


def source_hash():
    """Hash of everything that decides the measured kernel's traffic on this workload (the
    eval kernel's sources and the input generator); a stored traffic figure is used only
    while it matches."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2605_04550_amd", "csrc")
    for f in EVAL_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    h.update(open(os.path.join(ROOT, "workloads", "gen.py"), "rb").read())
    return h.hexdigest()[:16]


def summarize_counters(fetch_csv, write_csv):
    """HBM bytes per full-grid launch from two rocprofv3 --pmc runs of --counter-pass.  Each
    counter is scaled by what it reads for the calibration copy of known size (the first
    copy kernel of the run, CALIB_BYTES each way)."""
    import csv

    def rows(path, counter):
        out = []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
        return sorted(out)

    res = {}
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        rs = rows(path, counter)
        cid, calib = [(d, v) for d, k, v in rs if "copyBuffer" in k and v > 1000.0][0]
        # every library kernel of the full-grid call (the bisection kernel's two launches, the
        # list sort, the Golub-Kahan kernel)
        parts = {}
        for d, k, v in rs:
            if d > cid and "ps::" in k:
                name = k.split("(")[0].replace("void ", "")
                parts[name] = parts.get(name, 0.0) + v
        kern = sum(parts.values())
        factor = (CALIB_BYTES / 1024.0) / calib
        res[counter] = dict(kib=kern, calib_kib=calib, factor=factor, bytes=kern * 1024.0 * factor,
                            per_kernel_kib=parts)
    traffic = res["FETCH_SIZE"]["bytes"] + res["WRITE_SIZE"]["bytes"]
    doc = dict(kernel="full-grid call of toeplitz2000 (the bisection kernel ps::bis::k_bis<2, 2, 1, 1>, "
                      "ps::k_sort_lists, the Golub-Kahan kernel ps::k_eval<1, 1, false, false>)",
               source_hash=source_hash(), traffic_bytes_per_launch=traffic,
               fetch=res["FETCH_SIZE"], write=res["WRITE_SIZE"],
               commands=["timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/pmc_fetch "
                         "-o fetch -- python3 bench.py --workload toeplitz2000 --counter-pass",
                         "timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out>/pmc_write "
                         "-o write -- python3 bench.py --workload toeplitz2000 --counter-pass",
                         "python bench.py --workload toeplitz2000 --summarize-counters "
                         "<out>/pmc_fetch/fetch_counter_collection.csv <out>/pmc_write/write_counter_collection.csv"])
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print(json.dumps(doc, indent=1))


def stored_traffic():
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        doc = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if doc.get("source_hash") != source_hash():
        return None        # kernel or workload changed since the counters were taken
    return doc.get("traffic_bytes_per_launch")


def algorithmic_bytes(n, kl, ku, iters, info=None):
    """Bytes the method must move for one launch: the band once, and per Golub-Kahan shift
    the LU and its steps.  A shift that took the inertia bisection (info & 8) moves only its
    result: its passes read the band (cached) and keep the factor rows in registers."""
    wl, wu = kl, kl + ku + 1
    b_lu = (wl + wu) * 16 * n + n
    b_step = (2 * (wl + wu) + 10) * 16 * n + 2 * n
    iters = np.asarray(iters, dtype=np.float64)
    gk = np.ones(iters.shape, dtype=bool) if info is None else (np.asarray(info) & 8) == 0
    total = (kl + ku + 1) * 16 * n + np.sum(np.where(gk, b_lu + iters * b_step, 0.0) + 16)
    return float(total)


def tests_per_lane(hb, tests=0):
    """Tests per lane and bisection pass: the library's test-count modes (ps_opts.tests)."""
    if tests == 1:
        return 1
    if tests == 3:
        return 2 if hb <= 6 else 1
    return 3 if hb <= 2 else 2 if hb <= 5 else 1


def row_flops(hb, tests_per_pass):
    """FP64 operations of one row of a bisection pass (adds, multiplies, FMAs as executed, an FMA
    counting 2): forming the row of (zI-A)^H(zI-A) from the Gram band, 8 hb + 5, once per pass;
    per test the rank-one update of the trailing window (4 hb (hb - 1) off the diagonal), the
    scaled pivot column and the diagonal updates (6 hb), the shift and 1/pivot by the hardware
    reciprocal with two Newton steps (10)."""
    return 8 * hb + 5 + tests_per_pass * (4 * hb * (hb - 1) + 6 * hb + 10)


def bisection_flops(n, hb, info, lanes=1, tests=0):
    """Algorithmic floating-point operations of the bisection passes of one call: every pass
    covers all n rows; a pass of lanes * tests_per_lane tests forms the row of H once."""
    info = np.asarray(info, dtype=np.int64)
    passes = np.where((info & 8) != 0, info >> 8, 0).astype(np.float64)
    return float(np.sum(passes) * n * row_flops(hb, lanes * tests_per_lane(hb, tests)))


def _grid_points(grid):
    """Grid points of Sec. 2.1 in the library's convention (inclusive ends, row index <-> y)."""
    xs = np.array([grid.a + (grid.b - grid.a) * j / (grid.nx - 1) for j in range(grid.nx)])
    ys = np.array([grid.c + (grid.d - grid.c) * i / (grid.ny - 1) for i in range(grid.ny)])
    return (xs[None, :] + 1j * ys[:, None]).ravel()


def cpu_baseline(band, z_sample, threads):
    import oracle
    oracle.build(force=False)
    t = time.time()
    oracle.sigma_min(band, z_sample, nthreads=threads, parallel_pairs=True)
    dt = time.time() - t
    return dict(value=len(z_sample) / dt, unit="shifts/s", cores=threads, kind="oracle",
                sample="%d grid point(s) of the same workload (n=2000), dense one-sided Jacobi to convergence, "
                       "round-robin pairs over %d threads; %.1f s" % (len(z_sample), threads, dt))


def label_bench(args):
    """Label workload of Sec. 3.3: NMAT matrices (n = 64, eq. (matrix)), 100 x 100 grid on
    [-4, 4]^2, eps = 0.01, as one batch.  Times ps_label_batch (exclusion regions) against the
    plain method (ps_eval_batch on every point, labels sigma <= eps)."""
    import torch
    import workloads as W
    from paper_2605_04550_amd import api
    w = W.paper_label_workload(args.labels)
    grid, eps = w["grid"], w["eps"]
    mats = [api.BandedMatrix.from_band(b) for b in w["mats"]]
    batch = api.BandedBatch(mats, [grid] * len(mats))
    batch.label(eps)
    batch.eval(None)                          # warm-up of both paths
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        r = batch.label(eps)
    torch.cuda.synchronize()
    t_label = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        p = batch.eval(None)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / reps
    npts = grid.npts * len(mats)
    plain_lab = (p["sigma"] <= eps).to(torch.uint8)
    agree = int((plain_lab == r["label"]).sum().item())
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        threads = oracle.default_threads()
        zs = oracle.grid_points(grid)[:2000]
        t0 = time.perf_counter()
        oracle.sigma_min(w["mats"][0], zs, nthreads=threads)
        dt = time.perf_counter() - t0
        cpu = dict(value=len(zs) / dt, unit="points/s", cores=threads, kind="oracle",
                   sample="the plain method on the first 2000 grid points of matrix 0 (n=64): dense one-sided "
                          "Jacobi per point, points over %d threads; %.1f s" % (threads, dt))
    print(json.dumps({
        "metric": "grid points labelled per second (sensitive zone, eps = 0.01)", "value": npts / t_label,
        "unit": "points/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "Sec. 3.3 label workload: %d matrices n=64 (eq. (matrix)), 100x100 grid on "
                               "[-4,4]^2, one batch" % len(mats), "matrices": len(mats)},
        "label_s": t_label, "plain_s": t_plain, "plain_points_per_s": npts / t_plain,
        "speedup_vs_plain_method": t_plain / t_label,
        "evaluated_fraction": int(r["evals"].item()) / npts,
        "labels_equal_to_plain": agree, "points": npts, "cpu_baseline": cpu}), flush=True)


def trace_bench(args):
    """Contour tracing on the measured workload: args.trace seeds taken evenly from the
    eps = 1e-2 seeds of the full toeplitz2000 grid, traced inside the grid box with h = the
    grid spacing, 2 Newton steps per point, at most 64 points per tracer."""
    import torch
    import workloads as W
    from paper_2605_04550_amd import api
    w = W.workload("toeplitz2000")
    mat = api.BandedMatrix.from_band(w["band"])
    g = w["grid"]
    eps = EPS_ZONE
    r = api.eval_grid(mat, g)
    seeds, count = api.contour_seeds(g, r["sigma"], eps)
    pick = seeds[:: max(1, count // args.trace)][: args.trace].contiguous()
    h = (g.b - g.a) / (g.nx - 1)
    box = (g.a, g.b, g.c, g.d)
    api.trace_contour(mat, pick[:4], eps, h, 4, box=box)          # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr = api.trace_contour(mat, pick, eps, h, 64, box=box)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    npts = int(tr["count"].sum().item())
    fl = tr["flags"].cpu().numpy()
    print(json.dumps({
        "metric": "eps-contour points traced per second (predictor + 2 Newton steps, FP64)", "value": npts / dt,
        "unit": "points/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "toeplitz2000 eps=1e-2: %d seeds from the full-grid contour seeds, h = grid spacing, "
                               "<= 64 points each" % len(pick), "seeds": len(pick)},
        "seconds": dt, "points": npts,
        "flags": {"closed": int(np.sum(fl & 1 != 0)), "left_box": int(np.sum(fl & 2 != 0)),
                  "newton_failed": int(np.sum(fl & 4 != 0)), "max_points": int(np.sum(fl & 8 != 0))}}), flush=True)


# Network flops per evaluation of the classifier of Sec. 3.2: 2 x the multiply-adds its dense
# layers perform per point.  The 30 global-feature columns of the first matrix-path layer are
# folded into that layer's bias once per matrix (they do not depend on the point), so per point
# it multiplies only the g1..g3 columns: 26*64 + 64*64 + 3*128 + 128*64 + 2*128*128 + 128*64 + 64
# = 55 360 (59 200 with the folded columns).
MLP_FLOPS = 2 * 55360
FP32_MFMA_PEAK_TFLOPS = 157.3


def mask_bench(args):
    """The hybrid method of Sec. 4 on the Sec. 3.3 setting: NMAT matrices (n = 64, eq. (matrix)),
    100 x 100 grid on [-4, 4]^2.  Per matrix the mask producer (ps_mask_predict: classifier of
    Sec. 3.2 on the coarse grid of stride 4, refinement of the cells at or above the 80th
    percentile, tau = 0.05, 5 x 5 dilation; all matrices in one ps_mask_predict_batch call),
    then sigma_min on the masked points of all matrices in one ps_eval_batch call, against the
    plain method (every point).  The network is the one trained on exact labels of the same
    matrix class (paper_2605_04550_amd/train_mask.py; these matrices are held out from its
    training and validation sets) with its calibrated tau*, on the features of Sec. 3.1
    (paper_2605_04550_amd/features.py); recall of R and the sensitive points it misses are
    reported against the plain method's labels.  Also the classifier's throughput alone
    (ps_mlp_prob on 2^20 points) against the float32 matrix-core peak."""
    import torch
    import workloads as W
    from paper_2605_04550_amd import api
    from workloads import nets
    w = W.paper_label_workload(args.mask)
    grid = w["grid"]
    dev = torch.device("cuda:0")
    from paper_2605_04550_amd.features import band_features
    trained = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2605_04550_amd", "data", "mask_net.npz")
    if os.path.exists(trained):
        tw = np.load(trained, allow_pickle=False)
        net_params, tau = tw["params"], float(tw["tau"])
        weights = "trained (tau* %.2f)" % tau
    else:
        net_params, tau = nets.mlp_params(W.SEED_BASE + 900, 3.0), 0.05
        weights = "seeded draws (no trained weights found)"
    net = api.MaskNet(net_params)
    fe = [band_features(b, 3_000_000 + m) for m, b in enumerate(w["mats"])]
    eigs = [torch.tensor(lam, dtype=torch.complex128, device=dev) for _, lam in fe]
    gfs = [list(f) for f, _ in fe]
    mats = [api.BandedMatrix.from_band(b) for b in w["mats"]]
    batch = api.BandedBatch(mats, [grid] * len(mats))
    stream = torch.cuda.current_stream()

    def masks():
        return net.predict_batch(grid, gfs, eigs, tau=tau)

    rs = masks()
    batch.eval(list(rs["mask"]))
    batch.eval(None)
    net.predict(grid, gfs[0], eigs[0], tau=tau)
    torch.cuda.synchronize()
    reps = 3
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    t_mask = t_rest = 0.0
    for _ in range(reps):
        e0.record(stream)
        rs = masks()
        e1.record(stream)
        batch.eval(list(rs["mask"]))
        e2.record(stream)
        torch.cuda.synchronize()
        t_mask += e0.elapsed_time(e1) / 1e3 / reps
        t_rest += e1.elapsed_time(e2) / 1e3 / reps
    e0.record(stream)
    for _ in range(reps):
        batch.eval(None)
    e1.record(stream)
    torch.cuda.synchronize()
    t_plain = e0.elapsed_time(e1) / 1e3 / reps
    # one matrix alone (the single-matrix call's latency)
    e0.record(stream)
    for _ in range(reps):
        net.predict(grid, gfs[0], eigs[0], tau=tau)
    e1.record(stream)
    torch.cuda.synchronize()
    t_single = e0.elapsed_time(e1) / 1e3 / reps
    evals = int(rs["evals"].sum().item())
    region = int(rs["mask"].sum().item())
    npts = grid.npts * len(mats)
    # quality against the plain method's labels: recall of R (labels dilated 3 x 3, as in the
    # calibration of Sec. 3.6) and the sensitive points outside R (the hybrid's only errors)
    import scipy.ndimage as nd
    plain = batch.eval(None)
    lab = (plain["sigma"] <= 0.01).reshape(len(mats), grid.ny, grid.nx).cpu().numpy()
    rmask = rs["mask"].cpu().numpy().astype(bool)
    recalls, missed = [], 0
    for m in range(len(mats)):
        dl = nd.binary_dilation(lab[m], structure=np.ones((3, 3), dtype=bool))
        recalls.append(1.0 if dl.sum() == 0 else float((dl & rmask[m]).sum()) / float(dl.sum()))
        missed += int((lab[m] & ~rmask[m]).sum())
    # classifier throughput: 2^20 points of the grid box, one launch
    nthr = 1 << 20
    rng = np.random.default_rng(7)
    z = torch.tensor(rng.uniform(-4, 4, nthr) + 1j * rng.uniform(-4, 4, nthr), dtype=torch.complex128, device=dev)
    net.prob(gfs[0], eigs[0], z)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        net.prob(gfs[0], eigs[0], z)
    e1.record(stream)
    torch.cuda.synchronize()
    t_prob = e0.elapsed_time(e1) / 1e3 / reps
    achieved = MLP_FLOPS * nthr / t_prob / 1e12
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's hybrid method on matrix 0 (same weights, features and spectrum)
        import oracle
        from oracle import mask as OM
        oracle.build(force=False)
        threads = oracle.default_threads()
        t0 = time.perf_counter()
        om = OM.mask_predict(net_params, gfs[0], eigs[0].cpu().numpy(), grid, tau)
        region0 = np.flatnonzero(om["mask"].ravel())
        oracle.sigma_min(w["mats"][0], oracle.grid_points(grid)[region0], nthreads=threads)
        dt = time.perf_counter() - t0
        cpu = dict(value=grid.npts / dt, unit="points/s", cores=threads, kind="oracle",
                   sample="matrix 0: the oracle's mask (float64 network, %d evaluations) and dense Jacobi "
                          "sigma_min on its %d region points over %d threads; %.1f s"
                          % (om["evals"], len(region0), threads, dt))
    print(json.dumps({
        "metric": "grid points per second, hybrid method (mask producer + sigma_min on the mask)",
        "value": npts / (t_mask + t_rest), "unit": "points/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f32 (classifier) / f64 (sigma_min)", "data": "synthetic",
        "config": {"workload": "Sec. 3.3 setting: %d matrices n=64 (eq. (matrix)), 100x100 grid on [-4,4]^2, "
                               "stride 4, 80th percentile, 5x5 dilation, network: %s" % (len(mats), weights),
                   "matrices": len(mats), "tau": tau},
        "recall_median": float(np.median(recalls)), "recall_p10": float(np.percentile(recalls, 10)),
        "sensitive_points": int(lab.sum()), "sensitive_outside_region": missed,
        "mask_s": t_mask, "mask_ms_per_matrix": 1e3 * t_mask / len(mats), "mask_single_matrix_ms": 1e3 * t_single,
        "mask_evaluations_per_s": evals / t_mask, "restricted_eval_s": t_rest,
        "plain_s": t_plain, "speedup_vs_plain_method": t_plain / (t_mask + t_rest),
        "network_evaluations": evals, "evaluations_per_matrix": evals / len(mats),
        "region_fraction": region / npts,
        "classifier": {"points": nthr, "seconds": t_prob, "evaluations_per_s": nthr / t_prob,
                       "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFLOPS,
                                    "unit": "TFLOP/s", "frac": achieved / FP32_MFMA_PEAK_TFLOPS, "traffic": None,
                                    "kernel": "ps::mlp::k_points (one launch; + k_prep, 1 workgroup)",
                                    "algorithmic_flops_per_launch": MLP_FLOPS * nthr}},
        "cpu_baseline": cpu}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["batch64", "toeplitz2000", "random10k", "grcar4000"], default="batch64",
                    help="batch64 (default): the 64-matrix batch, the largest single-GPU configuration; "
                         "toeplitz2000: the n = 2000 full grid plus its annulus list; random10k: the n = 10^4 "
                         "random banded matrix on a 512 x 512 grid; grcar4000: Grcar n = 4000 with vectors, "
                         "the adjoint and Newton refinement of the contour seeds")
    ap.add_argument("--plain-shifts", type=int, default=64,
                    help="batch64: seeded shifts timed one per launch for the plain per-shift path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-points", type=int, default=1)
    ap.add_argument("--progress", action="store_true", help="synchronise and report after every timed step")
    ap.add_argument("--plain-points", type=int, default=32)
    ap.add_argument("--serial", action="store_true", help="run the full-grid and mask evaluations back to back")
    ap.add_argument("--counter-pass", action="store_true",
                    help="calibration copy + one full-grid call of the workload (with vectors for grcar4000), for rocprofv3 --pmc")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--lanes", type=int, choices=[1, 2, 4], default=None,
                    help="batch64, toeplitz2000: lanes per shift (with --tests: a fixed plan instead of the autotuned one; the "
                         "counter pass and its summary default to the library's default plan)")
    ap.add_argument("--tests", type=int, choices=[1, 2, 3], default=None,
                    help="batch64, toeplitz2000: tests-per-lane mode (see include/ps.h)")
    ap.add_argument("--trace", type=int, default=0, metavar="NSEED",
                    help="instead of the headline: trace the eps = 1e-2 contour of the workload from NSEED seeds")
    ap.add_argument("--labels", type=int, default=0, metavar="NMAT",
                    help="instead of the headline: label NMAT matrices of the Sec. 3.3 workload by exclusion "
                         "regions and by the plain method, one JSON line")
    ap.add_argument("--mask", type=int, default=0, metavar="NMAT",
                    help="instead of the headline: the hybrid method (mask producer + restricted sigma_min) on NMAT "
                         "matrices of the Sec. 3.3 setting, one JSON line")
    args = ap.parse_args()
    if args.summarize_counters:
        if args.workload == "batch64":
            summarize_batch_counters(*args.summarize_counters, lanes=args.lanes or 1, tests=args.tests or 2)
        else:
            summarize_counters(*args.summarize_counters)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(shifts are independent: several GPUs would each take their own share of them)", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2605_04550_amd import api

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.labels:
        label_bench(args)
        return
    if args.trace:
        trace_bench(args)
        return
    if args.mask:
        mask_bench(args)
        return
    if args.workload == "batch64":
        batch_bench(args, dev)
        return
    if args.workload == "random10k":
        random10k_bench(args, dev)
        return
    if args.workload == "grcar4000":
        grcar4000_bench(args, dev)
        return
    toeplitz_bench(args, dev)


BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batch64_traffic.json")
BATCH_SOURCES = ("ps_bisect.hpp", "ps_bisect.hip", "ps_internal.h", "ps_api.cpp") + tuple(
    "ps_bis_h%d.hip" % h for h in range(1, 9))


def batch_source_hash():
    """Hash of what decides the batch bisection kernel's traffic: its sources and the inputs."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2605_04550_amd", "csrc")
    for f in BATCH_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    h.update(open(os.path.join(ROOT, "workloads", "gen.py"), "rb").read())
    return h.hexdigest()[:16]


def batch_stored_traffic(lanes, tests):
    if not os.path.exists(BATCH_TRAFFIC_FILE):
        return None
    try:
        doc = json.load(open(BATCH_TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if doc.get("source_hash") != batch_source_hash():
        return None        # kernel or workload changed since the counters were taken
    if doc.get("plan", {"lanes": 1, "tests_mode": 2}) != {"lanes": lanes, "tests_mode": tests}:
        return None        # counters taken with another plan
    return doc.get("traffic_bytes_per_launch")


def summarize_batch_counters(fetch_csv, write_csv, lanes=1, tests=2):
    """HBM bytes of the bisection kernel's two launches in one batch call, from two rocprofv3
    --pmc runs of ``--counter-pass``, each counter scaled by its reading for the calibration
    copy of known size."""
    import csv

    def rows(path, counter):
        out = []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
        return sorted(out)

    res = {}
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        rs = rows(path, counter)
        cid, calib = [(d, v) for d, k, v in rs if "copyBuffer" in k and v > 1000.0][0]
        parts = [v for d, k, v in rs if d > cid and "k_bis<" in k]
        factor = (CALIB_BYTES / 1024.0) / calib
        res[counter] = dict(kib=sum(parts), launches=len(parts), calib_kib=calib, factor=factor,
                            bytes=sum(parts) * 1024.0 * factor)
    traffic = res["FETCH_SIZE"]["bytes"] + res["WRITE_SIZE"]["bytes"]
    doc = dict(kernel="ps::bis::k_bis<1, 8, %d, %d>, both launches of one batch64 call"
               % ({1: 0, 2: 1, 3: 2}[tests], lanes), plan={"lanes": lanes, "tests_mode": tests},
               source_hash=batch_source_hash(), traffic_bytes_per_launch=traffic,
               fetch=res["FETCH_SIZE"], write=res["WRITE_SIZE"],
               commands=["timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/pmc_fetch "
                         "-o fetch -- python3 bench.py --counter-pass --lanes %d --tests %d" % (lanes, tests),
                         "timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out>/pmc_write "
                         "-o write -- python3 bench.py --counter-pass --lanes %d --tests %d" % (lanes, tests),
                         "python bench.py --summarize-counters <out>/pmc_fetch/fetch_counter_collection.csv "
                         "<out>/pmc_write/write_counter_collection.csv --lanes %d --tests %d" % (lanes, tests)])
    with open(BATCH_TRAFFIC_FILE, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print(json.dumps(doc, indent=1))


def batch_bench(args, dev):
    """The headline: the 64-matrix batch (n ~ U{500..20000}, kl, ku ~ U{1..4}, CN(0,1) entries,
    128 x 128 grid on each matrix's Gershgorin box, 4915 masked points each: 314,560 shifts)
    through one ps_eval_batch call per step, captured once in a HIP graph and replayed."""
    import torch
    import workloads as W
    from paper_2605_04550_amd import api, ps_set_timing_events, ps_batch_workspace_size

    w = W.batch_workload()
    bands = [m["band"] for m in w["mats"]]
    mats = [api.BandedMatrix.from_band(b) for b in bands]
    batch = api.BandedBatch(mats, [m["grid"] for m in w["mats"]])
    masks = [torch.tensor(m["mask"], dtype=torch.uint8, device=dev).contiguous() for m in w["mats"]]
    mtab = batch.mask_table(masks, device=dev)
    if args.lanes is None and args.tests is None and not args.counter_pass:
        # the plan: lanes per shift and tests per lane chosen by timing the whole call
        # (ps_autotune_batch: one untimed call, then nine candidate plans, outside the timed region)
        tt = time.perf_counter()
        o = batch.autotune(mtab, device=dev)
        print("bench: autotuned plan lanes %d tests %d (%.1f s)" % (o.lanes, o.tests, time.perf_counter() - tt),
              file=sys.stderr, flush=True)
        tuned = True
    else:
        o = api.make_opts(lanes=args.lanes or 0, tests=args.tests or 0)
        tuned = False
    ws = torch.empty(ps_batch_workspace_size(batch.handle, o), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    nshift = int(sum(int(m["mask"].sum()) for m in w["mats"]))

    if args.counter_pass:
        x = torch.empty(CALIB_BYTES // 8, dtype=torch.float64, device=dev).fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print("bench: calibration copy done (%d bytes each way)" % CALIB_BYTES, file=sys.stderr, flush=True)
        del x, y
        batch.eval(mtab, workspace=ws, device=dev, opts=o)
        torch.cuda.synchronize()
        print("bench: batch call done", file=sys.stderr, flush=True)
        return

    stream = torch.cuda.Stream(device=dev)
    ev_s = torch.cuda.Event(enable_timing=True)
    ev_e = torch.cuda.Event(enable_timing=True)
    ev_s.record(stream)
    ev_e.record(stream)
    torch.cuda.synchronize()
    # eager warm-up (first-call set-up outside any timing), then one capture
    with torch.cuda.stream(stream):
        batch.eval(mtab, workspace=ws, device=dev, stream=stream, opts=o)
    torch.cuda.synchronize()
    print("bench: eager call done", file=sys.stderr, flush=True)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        out = batch.eval(mtab, workspace=ws, device=dev, stream=stream, opts=o)
    torch.cuda.synchronize()
    for i in range(args.warmup):
        graph.replay()
        torch.cuda.synchronize()
        print("bench: warmup replay %d done" % (i + 1), file=sys.stderr, flush=True)
    step_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        graph.replay()
        torch.cuda.synchronize()
        step_ms.append(1000.0 * (time.perf_counter() - ts))
        if args.progress:
            print("bench: replay %d done (%.1f s)" % (i + 1, time.perf_counter() - t0), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1000.0 * elapsed / args.steps
    value = nshift * args.steps / elapsed
    # the dominant kernel's duration: HIP events that the library records on the caller's
    # stream around its two bisection launches, on eager calls right after the timed replays
    bis_ms = []
    ps_set_timing_events(ev_s.cuda_event, ev_e.cuda_event)
    try:
        for i in range(3):
            with torch.cuda.stream(stream):
                batch.eval(mtab, workspace=ws, device=dev, stream=stream, opts=o)
            torch.cuda.synchronize()
            bis_ms.append(ev_s.elapsed_time(ev_e))
    finally:
        ps_set_timing_events(0, 0)

    # per-shift outcomes of the last replay
    counts = out["counts"].cpu().numpy()
    info = out["info"].cpu().numpy()
    iters = out["iters"].cpu().numpy()
    sig = out["sigma"].cpu().numpy()
    offs = out["offsets"]
    flops = 0.0
    gk_bytes = 0.0
    n_bis = n_gk = 0
    passes_all = []
    for m, b in enumerate(bands):
        sl = slice(offs[m], offs[m] + int(counts[m]))
        inf, it = info[sl], iters[sl]
        hb = b.kl + b.ku
        flops += bisection_flops(b.n, hb, inf, int(o.lanes) or 1, int(o.tests))
        bis = (inf & 8) != 0
        n_bis += int(bis.sum())
        n_gk += int((~bis).sum())
        passes_all.append(inf[bis] >> 8)
        gk_bytes += algorithmic_bytes(b.n, b.kl, b.ku, it, inf) - (b.kl + b.ku + 1) * 16 * b.n
    passes_all = np.concatenate(passes_all)
    dur_bis = float(np.median(bis_ms)) / 1000.0
    achieved = flops / dur_bis / 1e12
    traffic = batch_stored_traffic(int(o.lanes) or 1, int(o.tests) or 2)

    # plain per-shift GPU path: one wavefront per shift (lanes = 64: a pass tests 64 points of
    # the bracket), one call per shift driven from the host, no batching, no graph; timed on a
    # seeded sample of one masked shift per matrix, extrapolated matrix by matrix
    rng = np.random.default_rng(2605_04550 + 11)
    from paper_2605_04550_amd import ps_eval_points, ps_workspace_size
    op = api.make_opts(lanes=64)
    plain_total = 0.0
    plain_time = 0.0
    nplain = 0
    order = rng.permutation(len(bands))[:max(1, min(args.plain_shifts, len(bands)))]
    for m in order:
        b, mat = bands[m], mats[m]
        zs = _grid_points(w["mats"][m]["grid"])[rng.choice(np.flatnonzero(w["mats"][m]["mask"].ravel()))]
        z1 = torch.tensor([zs], dtype=torch.complex128, device=dev)
        ws1 = torch.empty(ps_workspace_size(mat.handle, 1, op), dtype=torch.uint8, device=dev)
        sig1 = torch.empty(1, dtype=torch.float64, device=dev)
        handle = torch.cuda.current_stream().cuda_stream
        torch.cuda.synchronize()
        tp = time.perf_counter()
        ps_eval_points(mat.handle, z1.data_ptr(), 1, op, ws1.data_ptr(), ws1.numel(), sig1.data_ptr(), 0, 0, 0, 0,
                       handle)
        torch.cuda.synchronize()
        dt = time.perf_counter() - tp
        plain_time += dt
        plain_total += dt * int(w["mats"][m]["mask"].sum())
        nplain += 1
    scale = nshift / sum(int(w["mats"][m]["mask"].sum()) for m in order)
    plain_total *= scale
    plain_value = nshift / plain_total

    out_line = {
        "metric": "shifts/sec sigma_min(zI-A) FP64 (|dsigma|<=1e-10||A||_F+1e-8 sigma)",
        "value": value,
        "unit": "shifts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "batch64: 64 banded matrices, n ~ U{500..20000}, kl, ku ~ U{1..4}, CN(0,1) entries, "
                        "128x128 grid on each Gershgorin box, 4915-point seeded mask each; one ps_eval_batch call "
                        "per step, replayed from a captured HIP graph",
            "matrices": len(bands), "shifts_per_step": nshift,
            "n_total": int(sum(b.n for b in bands)),
            "replay_ms_median": float(np.median(step_ms)), "replay_ms_min": float(np.min(step_ms)),
            "bisection_shifts": n_bis, "golub_kahan_shifts": n_gk,
            "bisection_passes_mean": float(passes_all.mean()) if passes_all.size else 0.0,
            "maxiter_shifts": int(np.sum((info[np.concatenate([np.arange(offs[m], offs[m] + counts[m]) for m in range(len(bands))])] & 2) != 0)),
            "plan": {"lanes": int(o.lanes) or 1, "tests_mode": int(o.tests) or 2, "autotuned": tuned,
                     "tests_modes": "1: one per lane; 2: 3 for kl+ku<=2, 2 for <=5, 1 above; "
                                    "3: 2 for kl+ku<=6, 1 above"},
        },
        "plain": {"value": plain_value, "unit": "shifts/s",
                  "sample": "%d seeded masked shifts, one per matrix, each one ps_eval_points call with "
                            "lanes = 64 (one wavefront per shift), host-driven, no graph; %.2f s measured, "
                            "extrapolated by each matrix's shift count" % (nplain, plain_time)},
        "speedup_vs_plain": value / plain_value,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": traffic,
            "kernel": "ps::bis::k_bis<1, 8, %d, %d> (inertia bisection, both launches of a call)"
                      % ({1: 0, 2: 1, 3: 2}[int(o.tests) or 2], int(o.lanes) or 1),
            "algorithmic_flops_per_launch": flops,
            "launch_ms_median": dur_bis * 1000.0,
            # the Golub-Kahan shifts run on side streams beside the bisection
            "golub_kahan_algorithmic_bytes": gk_bytes,
        },
    }
    if not args.no_cpu_baseline:
        # the oracle on a bounded sample: 32 seeded masked points of the smallest matrix,
        # one point per thread (dense one-sided Jacobi, cyclic pairs; about 17 s)
        k = int(np.argmin([b.n for b in bands]))
        rng2 = np.random.default_rng(2605_04550 + 12)
        cand = np.flatnonzero(w["mats"][k]["mask"].ravel())
        zs = _grid_points(w["mats"][k]["grid"])[rng2.choice(cand, size=32, replace=False)]
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        print("bench: timing the CPU oracle on %d points (n=%d)" % (len(zs), bands[k].n), file=sys.stderr,
              flush=True)
        import oracle
        oracle.build(force=False)
        tc = time.time()
        oracle.sigma_min(bands[k], zs, nthreads=threads, parallel_pairs=False)
        dtc = time.time() - tc
        ncube = np.array([b.n for b in bands], dtype=np.float64) ** 3
        per_shift = dtc / len(zs) / bands[k].n ** 3 * np.sum(ncube * 4915) / nshift
        out_line["cpu_baseline"] = dict(
            value=len(zs) / dtc, unit="shifts/s", cores=threads, kind="oracle",
            sample="%d seeded masked shifts of the smallest matrix of the batch (n=%d), dense one-sided Jacobi "
                   "to convergence, one shift per thread over %d threads; %.1f s" % (len(zs), bands[k].n, threads,
                                                                                      dtc),
            extrapolated_full_workload=dict(value=1.0 / per_shift if per_shift > 0 else None,
                                            unit="shifts/s", note="cost per shift scaled by n^3 to the batch's "
                                                                  "matrices; extrapolated, not measured"))
    print(json.dumps(out_line), flush=True)


def random10k_bench(args, dev):
    """Random banded n = 10^4 (kl = 2, ku = 3, CN(0,1)/sqrt(6) entries, diagonal + U[-1,1]) on a
    512 x 512 grid over its Gershgorin box: one full-grid ps_eval_grid call per step (262,144
    shifts), eager calls timed end to end; the bisection launches' duration from the library's
    timing hook; the roofline of the bisection kernel as for the headline."""
    import torch
    import workloads as W
    from paper_2605_04550_amd import api, ps_set_timing_events, ps_workspace_size
    w = W.workload("random10k")
    band, grid = w["band"], w["grid"]
    mat = api.BandedMatrix.from_band(band)
    o = api.make_opts()
    ws = torch.empty(ps_workspace_size(mat.handle, grid.npts, o), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    for i in range(max(1, args.warmup)):
        api.eval_grid(mat, grid, workspace=ws, device=dev)
        torch.cuda.synchronize()
        print("bench: warm-up call %d done" % (i + 1), file=sys.stderr, flush=True)
    ev_s, ev_e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev_s.record(stream)          # torch creates the underlying HIP events on their first record
    ev_e.record(stream)
    torch.cuda.synchronize()
    t_call, t_bis = [], []
    ps_set_timing_events(ev_s.cuda_event, ev_e.cuda_event)
    try:
        for i in range(args.steps):
            t0 = time.perf_counter()
            r = api.eval_grid(mat, grid, workspace=ws, device=dev)
            torch.cuda.synchronize()
            t_call.append(time.perf_counter() - t0)
            t_bis.append(ev_s.elapsed_time(ev_e) / 1e3)
            print("bench: call %d done (%.3f s)" % (i + 1, t_call[-1]), file=sys.stderr, flush=True)
    finally:
        ps_set_timing_events(0, 0)
    info = r["info"].cpu().numpy()
    flops = bisection_flops(band.n, band.kl + band.ku, info)
    bis = (info & 8) != 0
    tc, tb = float(np.median(t_call)), float(np.median(t_bis))
    achieved = flops / tb / 1e12
    print(json.dumps({
        "metric": "shifts/sec sigma_min(zI-A) FP64 (|dsigma|<=1e-10||A||_F+1e-8 sigma)",
        "value": grid.npts / tc, "unit": "shifts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * tc, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "random10k: random banded n=10^4, kl=2, ku=3, CN(0,1)/sqrt(6) + U[-1,1] diagonal, "
                               "512x512 grid on its Gershgorin box, one ps_eval_grid call per step (eager)",
                   "shifts_per_step": grid.npts, "bisection_shifts": int(bis.sum()),
                   "golub_kahan_shifts": int((~bis).sum()),
                   "bisection_passes_mean": float((info[bis] >> 8).mean()) if bis.any() else 0.0,
                   "maxiter_shifts": int(np.sum((info & 2) != 0))},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": "ps::bis::k_bis<5, 5, 1, 1> (both launches of a call)",
                     "algorithmic_flops_per_launch": flops, "launch_ms_median": 1e3 * tb},
        "cpu_baseline": None}), flush=True)


def grcar4000_bench(args, dev):
    """Grcar n = 4000 on a 256 x 256 grid over [-1.5, 3] x [-3.5, 3.5], the vectors-and-adjoint
    pipeline per step: sigma_min with both singular vectors at every grid point, the adjoint of
    L = sum_p w_p sigma_p (grad_z and the band gradient), the eps = 1e-3 contour seeds and three
    Newton steps from each.  Eager calls; the roofline is the adjoint's (it reads u and v, 2 x 16 n
    bytes per shift, once: HBM-bound)."""
    import torch
    import workloads as W
    from paper_2605_04550_amd import api
    w = W.workload("grcar4000")
    band, grid, eps = w["band"], w["grid"], w["eps"]
    band.real = False
    mat = api.BandedMatrix.from_band(band)
    wts = torch.tensor(w["weights"], device=dev)

    if args.counter_pass:
        # for rocprofv3 --pmc: a calibration copy of known size, then one grid call with vectors
        x = torch.empty(CALIB_BYTES // 8, dtype=torch.float64, device=dev).fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print("bench: calibration copy done (%d bytes each way)" % CALIB_BYTES, file=sys.stderr, flush=True)
        del x, y
        api.eval_grid(mat, grid, eps=eps, want_vectors=True, device=dev)
        torch.cuda.synchronize()
        print("bench: grid call with vectors done", file=sys.stderr, flush=True)
        return

    def step():
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record()
        r = api.eval_grid(mat, grid, eps=eps, want_vectors=True, device=dev)
        e[1].record()
        gz, gb = api.backward(mat, wts, r["u"], r["v"])
        e[2].record()
        seeds, count = api.contour_seeds(grid, r["sigma"], eps)
        z3, s3 = api.newton_contour(mat, seeds, eps, steps=3)
        e[3].record()
        torch.cuda.synchronize()
        return e, count
    for i in range(max(1, args.warmup)):
        step()
        print("bench: warm-up step %d done" % (i + 1), file=sys.stderr, flush=True)
    times = []
    for i in range(args.steps):
        t0 = time.perf_counter()
        e, count = step()
        times.append((time.perf_counter() - t0, e[0].elapsed_time(e[1]) / 1e3, e[1].elapsed_time(e[2]) / 1e3,
                      e[2].elapsed_time(e[3]) / 1e3))
        print("bench: step %d done (%.3f s)" % (i + 1, times[-1][0]), file=sys.stderr, flush=True)
    t = np.median(np.array(times), axis=0)
    adj_bytes = 2.0 * 16.0 * band.n * grid.npts + 16.0 * (band.kl + band.ku + 1) * band.n
    achieved = adj_bytes / t[2] / 1e9
    print(json.dumps({
        "metric": "shifts/sec sigma_min(zI-A) FP64 with singular vectors, adjoint and Newton refinement",
        "value": grid.npts / t[0], "unit": "shifts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * t[0], "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "grcar4000: Grcar n=4000, 256x256 grid on [-1.5,3]x[-3.5,3.5]; per step sigma with u, v "
                               "at every point, the adjoint of sum w_p sigma_p, eps=1e-3 contour seeds and 3 Newton "
                               "steps from each (eager calls)",
                   "shifts_per_step": grid.npts, "contour_seeds": int(count), "eval_ms": 1e3 * t[1],
                   "adjoint_ms": 1e3 * t[2], "seeds_newton_ms": 1e3 * t[3]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0,
                     "traffic": None, "kernel": "the adjoint (ps_backward: k_grad_z, k_grad_band_partial, "
                                                "k_grad_band_sum)",
                     "algorithmic_bytes_per_launch": adj_bytes},
        "cpu_baseline": None}), flush=True)


def toeplitz_bench(args, dev):
    """The toeplitz2000 line: full grid + annulus mask per step (see the module docstring)."""
    import torch
    import workloads as W
    from paper_2605_04550_amd import api
    w = W.workload("toeplitz2000")
    band, grid = w["band"], w["grid"]
    mat = api.BandedMatrix.from_band(band)
    mask = torch.tensor(w["mask"], dtype=torch.uint8, device=dev)
    npts_full = grid.npts
    npts_mask = int(w["mask"].sum())

    if args.counter_pass:
        x = torch.empty(CALIB_BYTES // 8, dtype=torch.float64, device=dev).fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print("bench: calibration copy done (%d bytes each way)" % CALIB_BYTES, file=sys.stderr, flush=True)
        del x, y
        r = api.eval_grid(mat, grid, eps=EPS_ZONE, device=dev)
        torch.cuda.synchronize()
        print("bench: full-grid launch done, iterations mean %.2f" % r["iters"].double().mean().item(),
              file=sys.stderr, flush=True)
        return

    # the plan: the library's default (one lane per shift, tests mode 2) unless --lanes / --tests
    # fix it.  Not autotuned: the tuner times a call alone, and the plans it picks for each call
    # of a step (two lanes for the full grid, four for the mask) make the step slower when the
    # two calls run together (13.1 against 12.1 ms)
    o = om = api.make_opts(lanes=args.lanes or 0, tests=args.tests or 0)
    tuned = False
    lanes, tests = int(o.lanes) or 1, int(o.tests) or 2
    lanes_m, tests_m = lanes, tests
    # workspaces allocated once, outside the timed region
    from paper_2605_04550_amd import ps_workspace_size
    ws = torch.empty(ps_workspace_size(mat.handle, npts_full, o), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    # The two evaluations of a step are independent: by default the restricted (mask) one
    # runs on a second stream with its own workspace, so its wavefronts take the SIMDs that
    # the full-grid launch frees as its short shifts finish.  --serial runs them one after
    # the other on one stream.
    stream_mask = stream if args.serial else torch.cuda.Stream(device=dev)
    ws_mask = ws if args.serial else torch.empty_like(ws)

    def step():
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        rf = api.eval_grid(mat, grid, eps=EPS_ZONE, workspace=ws, device=dev, stream=stream, lanes=lanes,
                           tests=tests)
        ev[1].record(stream)
        with torch.cuda.stream(stream_mask):
            stream_mask.wait_event(ev[0])
            ev[2].record(stream_mask)
            rm = api.eval_grid(mat, grid, mask, eps=EPS_ZONE, workspace=ws_mask, stream=stream_mask, lanes=lanes_m,
                               tests=tests_m)
            ev[3].record(stream_mask)
        stream.wait_event(ev[3])
        return rf, rm, ev

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print("bench: warmup step %d done" % (i + 1), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for i in range(args.steps):
        runs.append(step())
        if args.progress:
            torch.cuda.synchronize()
            print("bench: step %d done (%.1f s)" % (i + 1, time.perf_counter() - t0), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    ms_step = 1000.0 * elapsed / args.steps
    value = (npts_full + npts_mask) * args.steps / elapsed

    # roofline of the dominant kernel: the full-grid launch of the persistent kernel
    dur_full = np.mean([r[2][0].elapsed_time(r[2][1]) for r in runs]) / 1000.0
    dur_mask = np.mean([r[2][2].elapsed_time(r[2][3]) for r in runs]) / 1000.0
    rf, rm, _ = runs[-1]
    it_full = rf["iters"].cpu().numpy()
    info_full = rf["info"].cpu().numpy()
    cnt_mask = int(rm["count"].item())
    it_mask = rm["iters"][:cnt_mask].cpu().numpy()
    info_mask = rm["info"][:cnt_mask].cpu().numpy()
    bytes_full = algorithmic_bytes(band.n, band.kl, band.ku, it_full, info_full)
    achieved = bytes_full / dur_full / 1e9
    bytes_mask = algorithmic_bytes(band.n, band.kl, band.ku, it_mask, info_mask)
    si_full = (info_full & 8) != 0
    flops_full = bisection_flops(band.n, band.kl + band.ku, info_full)
    flops_mask = bisection_flops(band.n, band.kl + band.ku, info_mask)

    # plain per-shift GPU path (the speedup denominator): the same numerics and tolerance,
    # one launch per shift, no batching, on a seeded sample of the full grid
    rng = np.random.default_rng(2605_04550 + 7)
    sample = rng.choice(npts_full, size=args.plain_points, replace=False)
    zs_all = _grid_points(grid)
    z1 = torch.tensor(zs_all[sample], dtype=torch.complex128, device=dev)
    ws1 = torch.empty(ps_workspace_size(mat.handle, 1, o), dtype=torch.uint8, device=dev)
    sig1 = torch.empty(1, dtype=torch.float64, device=dev)
    from paper_2605_04550_amd import ps_eval_points
    handle = stream.cuda_stream
    ps_eval_points(mat.handle, z1[0:1].data_ptr(), 1, o, ws1.data_ptr(), ws1.numel(), sig1.data_ptr(), 0, 0, 0, 0,
                   handle)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for p in range(args.plain_points):
        ps_eval_points(mat.handle, z1[p:p + 1].data_ptr(), 1, o, ws1.data_ptr(), ws1.numel(), sig1.data_ptr(), 0, 0,
                       0, 0, handle)
    torch.cuda.synchronize()
    plain_value = args.plain_points / (time.perf_counter() - tp0)

    traffic = stored_traffic()

    out = {
        "metric": "shifts/sec sigma_min(zI-A) FP64 (|dsigma|<=1e-10||A||_F+1e-8 sigma)",
        "value": value,
        "unit": "shifts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "toeplitz2000: tridiagonal Toeplitz n=2000 (0.25, 0, 1), 256x256 grid on [-2,2]^2, "
                        "full grid + 25% annulus mask per step",
            "n": band.n, "kl": band.kl, "ku": band.ku,
            "shifts_per_step": npts_full + npts_mask,
            "full_grid_ms": dur_full * 1000.0, "mask_ms": dur_mask * 1000.0,
            "mask_stream": "serial" if args.serial else "concurrent",
            "iters_mean_full": float(it_full.mean()), "iters_max_full": int(it_full.max()),
            "iters_mean_mask": float(it_mask.mean()) if cnt_mask else 0.0,
            "maxiter_points_full": int(np.sum((info_full & 2) != 0)),
            "bisection_points_full": int(si_full.sum()),
            "bisection_passes_mean": float((info_full[si_full] >> 8).mean()) if si_full.any() else 0.0,
            "plan": {"lanes": lanes, "tests_mode": tests, "autotuned": tuned},
        },
        "plain": {"value": plain_value, "unit": "shifts/s",
                  "sample": "%d seeded points of the full grid, one launch per shift (same kernel numerics and "
                            "tolerance, no batching)" % args.plain_points},
        "speedup_vs_plain": value / plain_value,
        "roofline": {
            "bound": "alu",
            "achieved": flops_full / dur_full / 1e12,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": flops_full / dur_full / 1e12 / FP64_PEAK_TFLOPS,
            "traffic": traffic,
            "kernel": "full-grid call: the bisection kernel ps::bis::k_bis (first pass, then resumed) and the "
                      "Golub-Kahan kernel ps::k_eval<1,1,false,false> beside it on a side stream",
            "algorithmic_flops_per_launch": flops_full,
            # bytes of the Golub-Kahan shifts and of the outputs, and the HBM rate they make
            "algorithmic_bytes_per_launch": bytes_full,
            "hbm_achieved_gbs": achieved,
            # both launches of a step (they overlap unless --serial) over the step time
            "step_algorithmic_flops": flops_full + flops_mask,
            "step_achieved": (flops_full + flops_mask) / (ms_step / 1000.0) / 1e12,
        },
    }
    if not args.no_cpu_baseline:
        rng = np.random.default_rng(2605_04550)
        zs = _grid_points(grid)[rng.choice(npts_full, size=args.cpu_points, replace=False)]
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        print("bench: timing the CPU oracle on %d point(s)" % len(zs), file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(band, zs, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
