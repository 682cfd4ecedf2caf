"""GPU tests of the batch path (ps_create_batch / ps_eval_batch): many matrices of uneven n
and bandwidth, each with its own grid and mask, in one call."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import certify, column_norm_bound, golden, johnson_bound, need_gpu, report, tol

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


def _batch64(api, torch):
    w = W.batch_workload()
    mats = [api.BandedMatrix.from_band(m["band"]) for m in w["mats"]]
    batch = api.BandedBatch(mats, [m["grid"] for m in w["mats"]])
    masks = [torch.tensor(m["mask"], device="cuda").contiguous() for m in w["mats"]]
    return w, mats, batch, masks


def test_batch64_full_workload_certified():
    """The 64-matrix workload (n in [500, 20000], kl, ku in 1..4, 128x128 grids, 4915-point
    masks) in one ps_eval_batch call, as the benchmark makes it.  Every shift: finite, no
    MAXITER, 1-Lipschitz between masked grid neighbours; stored oracle values (two per matrix
    with n <= 5000); per matrix an inertia certificate on 8 shifts stratified by sigma and
    Johnson's lower bound and the column-norm upper bound on 64 seeded shifts."""
    api = _api()
    import time
    import torch
    w, mats, batch, masks = _batch64(api, torch)
    print("batch64: launching %d matrices, %d shifts" % (len(mats), 64 * 4915), flush=True)
    t = time.perf_counter()
    r = batch.eval(masks)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    counts = r["counts"].cpu().numpy()
    assert np.all(counts == 4915)
    sig = r["sigma"].cpu().numpy()
    info = r["info"].cpu().numpy()
    idx = r["idx"].cpu().numpy()
    sel = np.concatenate([np.arange(o, o + 4915) for o in r["offsets"]])
    assert np.all(np.isfinite(sig[sel])) and np.all(sig[sel] >= 0)
    assert np.all((info[sel] & 2) == 0), "MAXITER at %d shifts" % np.sum((info[sel] & 2) != 0)
    print("batch64: %d shifts in %.3f s (first call, with set-up); bisection at %d shifts"
          % (len(sel), dt, np.sum((info[sel] & 8) != 0)), flush=True)
    rng = np.random.default_rng(2605)
    for m, mm in enumerate(w["mats"]):
        b, g = mm["band"], mm["grid"]
        off = r["offsets"][m]
        im = idx[off:off + 4915]
        assert np.array_equal(im, oracle.compact_mask(mm["mask"]))
        sm = sig[off:off + 4915]
        zs = oracle.grid_points(g)[im]
        bnd = tol(b.fro, sm)
        # 1-Lipschitz between masked neighbours (full grid of sigma with NaN outside the mask)
        S = np.full(g.npts, np.nan)
        S[im] = sm
        S = S.reshape(g.ny, g.nx)
        B = np.full(g.npts, np.nan)
        B[im] = bnd
        B = B.reshape(g.ny, g.nx)
        hx = (g.b - g.a) / (g.nx - 1)
        hy = (g.d - g.c) / (g.ny - 1)
        for dS, dB, h in [(S[:, 1:] - S[:, :-1], B[:, 1:] + B[:, :-1], hx), (S[1:] - S[:-1], B[1:] + B[:-1], hy)]:
            ok = np.isnan(dS) | (np.abs(dS) <= h * (1 + 1e-12) + dB)
            assert ok.all(), (m, np.nanmax(np.abs(dS) - h - dB))
        pick = rng.choice(4915, 64, replace=False)
        assert np.all(sm[pick] >= johnson_bound(b, zs[pick]) - bnd[pick]), m
        assert np.all(sm[pick] <= column_norm_bound(b, zs[pick]) * (1 + 1e-12) + bnd[pick]), m
        # 8 shifts stratified by sigma among those the count can certify (sigma >= 1e-3)
        order = np.argsort(sm)
        order = order[sm[order] >= 1e-3]
        strat = order[np.unique(np.linspace(0, len(order) - 1, 8).astype(int))]
        assert len(strat) == 8, m
        certify(b, zs[strat], sm[strat], bnd[strat], "batch64 matrix %d (n=%d kl=%d ku=%d)" % (m, b.n, b.kl, b.ku))
    g = golden("batch_pts")
    for mi, k, zz, s_or in zip(g["mat"], g["idx"], g["z"], g["sigma"]):
        off = r["offsets"][mi]
        pos = np.searchsorted(idx[off:off + 4915], k)
        assert idx[off + pos] == k
        got = sig[off + pos]
        b = tol(w["mats"][mi]["band"].fro, s_or)
        assert abs(got - s_or) <= b, (mi, k, got, s_or)
    print("batch64: %d stored oracle points within the bar" % len(g["sigma"]), flush=True)


def test_batch64_graph_replays_match_eager():
    """The full 64-matrix call captured in a HIP graph: three replays, each with eager work and
    synchronisation between them, equal to the eager result bit for bit."""
    api = _api()
    import torch
    w, mats, batch, masks = _batch64(api, torch)
    mtab = batch.mask_table(masks)
    eager = batch.eval(mtab)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.eval(mtab, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        got = batch.eval(mtab)
    # the masked positions of every matrix (the others are never written)
    sel = torch.tensor(np.concatenate([np.arange(o, o + 4915) for o in eager["offsets"]]), device="cuda")
    for rep in range(3):
        got["sigma"].fill_(-1.0)
        got["info"].fill_(-1)
        x = torch.ones(1 << 20, device="cuda").sum()          # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert float(x) == float(1 << 20)
        assert torch.equal(got["counts"], eager["counts"]), rep
        assert torch.equal(got["sigma"][sel], eager["sigma"][sel]), rep
        assert torch.equal(got["info"][sel], eager["info"][sel]), rep
    print("batch64: 3 graph replays identical to the eager call", flush=True)
