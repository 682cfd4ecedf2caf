"""GPU tests of the batch path (ps_create_batch / ps_eval_batch): many matrices of uneven n
and bandwidth, each with its own grid and mask, in one call."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import golden, need_gpu, report, tol

pytestmark = pytest.mark.gpu


def _api():
    need_gpu()
    from paper_2605_04550_amd import api
    return api


def test_small_mixed_batch_matches_single_matrix_path_and_oracle():
    api = _api()
    import torch
    rng = np.random.default_rng(41)
    specs = [(130, 1, 2), (257, 2, 1), (64, 1, 2), (300, 0, 3), (97, 3, 0), (211, 4, 4), (50, 2, 2)]
    bands, grids, masks, mats = [], [], [], []
    for m, (n, kl, ku) in enumerate(specs):
        b = W.random_banded(n, kl, ku, seed=500 + m)
        a, bb, c, d = W.gershgorin_box(b)
        g = W.Grid(a, bb, c, d, 13 + m, 9 + 2 * m)     # ragged sizes
        bands.append(b)
        grids.append(g)
        mats.append(api.BandedMatrix.from_band(b))
        if m % 3 == 2:
            masks.append(None)                          # full grid
        else:
            masks.append(torch.tensor((rng.uniform(size=(g.ny, g.nx)) < 0.4).astype(np.uint8), device="cuda"))
    batch = api.BandedBatch(mats, grids)
    r = batch.eval(masks)
    torch.cuda.synchronize()
    counts = r["counts"].cpu().numpy()
    idx = r["idx"].cpu().numpy()
    sig = r["sigma"].cpu().numpy()
    info = r["info"].cpu().numpy()
    for m, (b, g) in enumerate(zip(bands, grids)):
        off = r["offsets"][m]
        exp_idx = np.arange(g.npts) if masks[m] is None else oracle.compact_mask(masks[m].cpu().numpy())
        assert counts[m] == len(exp_idx)
        assert np.array_equal(idx[off:off + counts[m]], exp_idx)
        z = oracle.grid_points(g)[exp_idx]
        single = api.sigma_min(mats[m], torch.tensor(z, dtype=torch.complex128, device="cuda"))
        s1 = single["sigma"].cpu().numpy()
        sb = sig[off:off + counts[m]]
        # same arithmetic in both paths: equal to rounding
        np.testing.assert_allclose(sb, s1, rtol=1e-13, atol=0)
        assert np.all((info[off:off + counts[m]] & 2) == 0)
        pick = np.arange(0, len(z), max(1, len(z) // 5))
        ref = oracle.sigma_min(b, z[pick])["sigma"]
        bnd = tol(b.fro, ref)
        report("batch matrix %d (n=%d kl=%d ku=%d)" % (m, b.n, b.kl, b.ku), sb[pick], ref, bnd)
        assert np.all(np.abs(sb[pick] - ref) <= bnd)


def test_batch64_workload_runs_and_matches_stored_oracle_points():
    """The 64-matrix workload (n in [500, 20000], kl, ku in 1..4, 128x128 grids, 4915-point
    masks) through one ps_eval_batch call; stored oracle values for the matrices with n <= 1200."""
    api = _api()
    import time
    import torch
    w = W.batch_workload()
    mats = [api.BandedMatrix.from_band(m["band"]) for m in w["mats"]]
    batch = api.BandedBatch(mats, [m["grid"] for m in w["mats"]])
    masks = [torch.tensor(m["mask"], device="cuda") for m in w["mats"]]
    print("batch64: launching %d matrices, %d shifts" % (len(mats), 64 * 4915), flush=True)
    t = time.perf_counter()
    r = batch.eval(masks)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    counts = r["counts"].cpu().numpy()
    assert np.all(counts == 4915)
    sig = r["sigma"].cpu().numpy()
    info = r["info"].cpu().numpy()
    it = r["iters"].cpu().numpy()
    sel = np.concatenate([np.arange(o, o + 4915) for o in r["offsets"]])
    assert np.all(np.isfinite(sig[sel])) and np.all(sig[sel] >= 0)
    print("batch64: %d shifts in %.3f s = %.0f shifts/s (first call, with set-up); Golub-Kahan steps mean %.1f "
          "max %d; bisection at %d shifts; MAXITER %d"
          % (len(sel), dt, len(sel) / dt, it[sel].mean(), it[sel].max(), np.sum((info[sel] & 8) != 0),
             np.sum((info[sel] & 2) != 0)), flush=True)
    g = golden("batch_pts")
    for mi, k, zz, s_or in zip(g["mat"], g["idx"], g["z"], g["sigma"]):
        off = r["offsets"][mi]
        pos = np.searchsorted(r["idx"][off:off + 4915].cpu().numpy(), k)
        got = sig[off + pos]
        b = tol(w["mats"][mi]["band"].fro, s_or)
        assert abs(got - s_or) <= b, (mi, k, got, s_or)
