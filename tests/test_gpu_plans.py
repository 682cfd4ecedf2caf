"""GPU parity of every plan of the inertia bisection.  Lanes per shift (1, 2, 4, or 64: a
wavefront per shift) and tests per lane (modes 1, 2, 3) select distinct instantiations of the
bisection kernel, and the tuners may pick any of them; each must give sigma within the parity
bar of the oracle.  Single-matrix calls at half-bandwidths kl + ku = 1, 2, 5, 8; the batch
kernel with lanes 1, 2, 4 and every test mode on a small mixed batch, against the same shifts
through the single-matrix path."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import need_gpu, report, tol

pytestmark = pytest.mark.gpu

PLANS = [(lanes, tests) for lanes in (1, 2, 4, 64) for tests in (1, 2, 3)]


def test_every_single_matrix_plan_matches_oracle():
    torch = need_gpu()
    from paper_2605_04550_amd import api
    shapes = [(240, 1, 0), (240, 1, 1), (200, 2, 3), (160, 4, 4)]
    for k, (n, kl, ku) in enumerate(shapes):
        band = W.random_banded(n, kl, ku, seed=1300 + k)
        a, b, c, d = W.gershgorin_box(band)
        rng = np.random.default_rng(130 + k)
        z = rng.uniform(a, b, 16) + 1j * rng.uniform(c, d, 16)
        ref = oracle.sigma_min(band, z)["sigma"]
        bnd = tol(band.fro, ref)
        mat = api.BandedMatrix.from_band(band)
        zt = torch.tensor(z, dtype=torch.complex128, device="cuda")
        passes = {}
        for lanes, tests in PLANS:
            print("shape n=%d kl=%d ku=%d plan lanes %d tests %d" % (n, kl, ku, lanes, tests), flush=True)
            r = api.sigma_min(mat, zt, lanes=lanes, tests=tests)
            s = r["sigma"].cpu().numpy()
            info = r["info"].cpu().numpy()
            assert np.all((info & 2) == 0), (kl, ku, lanes, tests)
            err = np.abs(s - ref)
            if not np.all(err <= bnd):
                report("kl=%d ku=%d lanes %d tests %d" % (kl, ku, lanes, tests), s, ref, bnd)
            assert np.all(err <= bnd), (kl, ku, lanes, tests, np.flatnonzero(err > bnd).tolist())
            used = (info & 8) != 0
            assert used.sum() >= 8, (kl, ku, lanes, tests, int(used.sum()))
            passes[(lanes, tests)] = (info[used] >> 8).mean()
        # more test points per pass take fewer passes: a wavefront per shift (64 points a pass)
        # against one point a pass
        print("kl=%d ku=%d passes: %s" % (kl, ku, {p: round(float(v), 1) for p, v in passes.items()}), flush=True)
        assert passes[(64, 1)] < passes[(1, 1)]


def test_every_batch_plan_matches_single_matrix_path():
    torch = need_gpu()
    from paper_2605_04550_amd import api
    rng = np.random.default_rng(1410)
    specs = [(150, 1, 0), (120, 1, 1), (90, 2, 3), (70, 4, 4), (110, 0, 2)]
    bands, grids, masks, mats = [], [], [], []
    for m, (n, kl, ku) in enumerate(specs):
        b = W.random_banded(n, kl, ku, seed=1400 + m)
        a, bb, c, d = W.gershgorin_box(b)
        g = W.Grid(a, bb, c, d, 11 + m, 7 + 2 * m)
        bands.append(b)
        grids.append(g)
        mats.append(api.BandedMatrix.from_band(b))
        masks.append(torch.tensor((rng.uniform(size=(g.ny, g.nx)) < 0.5).astype(np.uint8), device="cuda"))
    batch = api.BandedBatch(mats, grids)
    # the same shifts through the single-matrix path (default plan): pinned to the oracle by
    # the parity tests, and here at a few points per matrix
    single = []
    for m, (b, g) in enumerate(zip(bands, grids)):
        z = oracle.grid_points(g)[oracle.compact_mask(masks[m].cpu().numpy())]
        s1 = api.sigma_min(mats[m], torch.tensor(z, dtype=torch.complex128, device="cuda"))["sigma"].cpu().numpy()
        pick = np.arange(0, len(z), max(1, len(z) // 4))
        ref = oracle.sigma_min(b, z[pick])["sigma"]
        assert np.all(np.abs(s1[pick] - ref) <= tol(b.fro, ref)), m
        single.append(s1)
    for lanes in (1, 2, 4):
        for tests in (1, 2, 3):
            print("batch plan lanes %d tests %d" % (lanes, tests), flush=True)
            r = batch.eval(masks, lanes=lanes, tests=tests)
            torch.cuda.synchronize()
            counts = r["counts"].cpu().numpy()
            sig = r["sigma"].cpu().numpy()
            info = r["info"].cpu().numpy()
            nbis = 0
            for m, b in enumerate(bands):
                off = r["offsets"][m]
                assert counts[m] == len(single[m])
                sb = sig[off:off + counts[m]]
                ib = info[off:off + counts[m]]
                assert np.all((ib & 2) == 0), (m, lanes, tests)
                # both within the bar of the true sigma: within twice the bar of each other
                assert np.all(np.abs(sb - single[m]) <= 2 * tol(b.fro, single[m])), (m, lanes, tests)
                nbis += int(((ib & 8) != 0).sum())
            assert nbis >= int(counts.sum()) // 2, (lanes, tests, nbis)
