"""Writes the stored expected values used by the GPU parity tests.

Every number written here comes from the CPU oracle (``oracle/``) evaluated on
the seeded inputs of ``workloads``; nothing is read back from the GPU library.

    python tests/golden/make_golden.py [set ...] [--threads T]

Sets (file ``tests/golden/<set>.npz``):
  grcar100_all       Grcar n=100, 64x64 grid on [-1.5,3]x[-3.5,3.5]: all 4096 points.
  toeplitz2000_pts   Tridiagonal Toeplitz n=2000 (0.25, 0, 1): 8 full-grid points stratified
                     inside / near / outside the symbol ellipse, plus 8 points of the
                     restricted annulus list.
  random1000_grid    Replica of the random banded workload at n=1000 (same generator,
                     kl=2, ku=3, CN(0,1)/sqrt(6), diagonal + U[-1,1]): 16x16 grid on its
                     Gershgorin box, all 256 points.
  grcar400_vec       Grcar n=400, 32 seeded points of the 256x256 grid on [-1.5,3]x[-3.5,3.5],
                     with singular vectors and the two smallest singular values.
  batch_pts          Two seeded masked points for each matrix of the 64-matrix batch with
                     n <= 5000 (14 matrices).
  grcar4000_grad     Grcar n=4000 (the vectors-and-adjoint workload): 32 seeded grid points with
                     1e-8 <= sigma < 1 and sigma_{n-1} >= 1.05 sigma_n, their singular pairs from
                     LAPACK's dense SVD, and the gradients of L = sum_p w_p sigma_p (w the
                     workload's weights at those points): grad_z [32] and the band gradient
                     [n, kl+ku+1] (GB layout, complex: no real projection).
  paper_labels       The first three matrices of the label workload of Sec. 3.3 (n = 64,
                     100x100 grid on [-4,4]^2): sigma at all 10^4 points and the labels
                     sigma <= 0.01 (keys sigma0.., label0..).
Each file holds: idx (flat grid index, or -1), z, sigma, s2 (second smallest singular
value), and where stated u, v.
"""
import argparse
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def _two_smallest(sall):
    s = np.sort(sall, axis=1)
    return s[:, 0], s[:, 1]


def _save(name, **arrays):
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, **arrays)
    print("wrote", path, {k: v.shape for k, v in arrays.items()}, flush=True)


def grcar100_all(threads):
    w = W.workload("grcar100")
    z = oracle.grid_points(w["grid"])
    r = oracle.sigma_min(w["band"], z, all_sv=True, nthreads=threads, parallel_pairs=False)
    s1, s2 = _two_smallest(r["sall"])
    _save("grcar100_all", idx=np.arange(z.size), z=z, sigma=r["sigma"], s2=s2)


def toeplitz2000_pts(threads):
    w = W.workload("toeplitz2000")
    z = oracle.grid_points(w["grid"])
    re = np.sqrt((z.real / 1.25) ** 2 + (z.imag / 0.75) ** 2)   # elliptic radius of the symbol curve
    rng = np.random.default_rng(W.SEED_BASE + 102)
    pick = []
    for sel, cnt in [(re < 0.9, 3), ((re >= 0.9) & (re <= 1.1), 2), (re > 1.1, 3)]:
        pick += list(rng.choice(np.flatnonzero(sel), size=cnt, replace=False))
    pick += list(rng.choice(w["list"], size=8, replace=False))
    idx = np.array(pick, dtype=np.int64)
    zz = z[idx]
    r = oracle.sigma_min(w["band"], zz, all_sv=True, nthreads=threads, parallel_pairs=True)
    s1, s2 = _two_smallest(r["sall"])
    _save("toeplitz2000_pts", idx=idx, z=zz, sigma=r["sigma"], s2=s2)


def random1000_band():
    return W.random_banded(1000, 2, 3, W.SEED_BASE + 3, scale=1.0 / math.sqrt(6.0), diag_uniform=1.0)


def random1000_grid(threads):
    band = random1000_band()
    a, b, c, d = W.gershgorin_box(band)
    grid = W.Grid(a, b, c, d, 16, 16)
    z = oracle.grid_points(grid)
    r = oracle.sigma_min(band, z, all_sv=True, nthreads=threads, parallel_pairs=False)
    s1, s2 = _two_smallest(r["sall"])
    _save("random1000_grid", idx=np.arange(z.size), z=z, sigma=r["sigma"], s2=s2,
          box=np.array([a, b, c, d]))


def grcar400_vec(threads):
    band = W.grcar(400)
    grid = W.Grid(-1.5, 3.0, -3.5, 3.5, 256, 256)
    z = oracle.grid_points(grid)
    rng = np.random.default_rng(W.SEED_BASE + 105)
    idx = np.sort(rng.choice(z.size, size=32, replace=False)).astype(np.int64)
    r = oracle.sigma_min(band, z[idx], want_vectors=True, all_sv=True, nthreads=threads,
                         parallel_pairs=False)
    s1, s2 = _two_smallest(r["sall"])
    _save("grcar400_vec", idx=idx, z=z[idx], sigma=r["sigma"], s2=s2, u=r["u"], v=r["v"])


def batch_pts(threads):
    w = W.batch_workload()
    rng = np.random.default_rng(W.SEED_BASE + 104)
    rows = []
    for m, mat in enumerate(w["mats"]):
        if mat["band"].n > 5000:
            continue
        cand = oracle.compact_mask(mat["mask"])
        for k in np.sort(rng.choice(cand, size=2, replace=False)):
            zz = oracle.grid_points(mat["grid"])[int(k)]
            t = time.time()
            r = oracle.sigma_min(mat["band"], [zz], all_sv=True, nthreads=threads, parallel_pairs=True)
            s1, s2 = _two_smallest(r["sall"])
            rows.append((m, int(k), zz, r["sigma"][0], s2[0]))
            print("batch matrix", m, "n", mat["band"].n, "point", int(k), "%.0f s" % (time.time() - t), flush=True)
    m, k, zz, s, s2 = map(np.array, zip(*rows))
    _save("batch_pts", mat=m.astype(np.int64), idx=k.astype(np.int64), z=zz.astype(complex), sigma=s, s2=s2)


def paper_labels(threads):
    w = W.paper_label_workload(3)
    z = oracle.grid_points(w["grid"])
    out = {}
    for m, band in enumerate(w["mats"]):
        r = oracle.sigma_min(band, z, nthreads=threads, parallel_pairs=False)
        out["sigma%d" % m] = r["sigma"]
        out["label%d" % m] = oracle.sensitive(r["sigma"], w["eps"])
        print("paper-class matrix", m, "beta", band.kl, "sensitive", int(out["label%d" % m].sum()), flush=True)
    _save("paper_labels", **out)


def grcar4000_grad(threads):
    w = W.workload("grcar4000")
    band = w["band"]
    z = oracle.grid_points(w["grid"])
    rng = np.random.default_rng(W.SEED_BASE + 107)
    rows = []
    for k in rng.permutation(z.size):
        zz = z[k:k + 1]
        # Before the dense SVD (which decides): sigma_min in [1e-8, 1) and sigma_{n-1} >= 1.05
        # sigma_min by inertia counts (sigma_min bracketed by bisection on the count, then one
        # count at 1.05 times its upper end).  The counts are not trusted where sigma_min is
        # far below 1e-8 (deep inside the pseudospectrum of this matrix), hence the SVD check.
        cnt = lambda t: oracle.count_below(band, zz, t, threads)[0]
        if cnt(1.0) < 1 or cnt(1e-8) != 0:
            continue
        lo, hi = 1e-8, 1.0
        for _ in range(30):
            mid = math.sqrt(lo * hi)
            lo, hi = (lo, mid) if cnt(mid) >= 1 else (mid, hi)
        if hi < 1e-7 or cnt(1.05 * hi) != 1:
            continue
        t = time.time()
        r = oracle.smallest_pair_lapack(band, zz)
        ok = r["s2"][0] >= 1.05 * r["sigma"][0] and 1e-8 <= r["sigma"][0] < 1.0
        print("grcar4000 point", int(k), "sigma %.3e gap %.3f" % (r["sigma"][0], r["s2"][0] / r["sigma"][0]),
              "kept" if ok else "skipped", "%.0f s" % (time.time() - t), flush=True)
        if ok:
            rows.append((int(k), r))
        if len(rows) == 32:
            break
    idx = np.array([k for k, _ in rows], dtype=np.int64)
    u = np.concatenate([r["u"] for _, r in rows])
    v = np.concatenate([r["v"] for _, r in rows])
    wts = w["weights"][idx]
    gz, gb = oracle.adjoint(band, u, v, wts)
    _save("grcar4000_grad", idx=idx, z=z[idx], sigma=np.array([r["sigma"][0] for _, r in rows]),
          s2=np.array([r["s2"][0] for _, r in rows]), grad_z=gz, grad_band=gb)


SETS = dict(grcar100_all=grcar100_all, toeplitz2000_pts=toeplitz2000_pts, random1000_grid=random1000_grid,
            grcar400_vec=grcar400_vec, batch_pts=batch_pts, paper_labels=paper_labels, grcar4000_grad=grcar4000_grad)

if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("sets", nargs="*", default=list(SETS))
    ap.add_argument("--threads", type=int, default=oracle.default_threads())
    args = ap.parse_args()
    oracle.build(force=False)
    for s in args.sets:
        t = time.time()
        SETS[s](args.threads)
        print(s, "done in %.1f s" % (time.time() - t), flush=True)
