"""GPU tests of the exclusion-region labelling (ps_label_grid): the sensitive zone of
Sec. 2.1 on the label workload of Sec. 3.3 (n = 64 matrices of the class of eq. (matrix),
100 x 100 grid on [-4, 4]^2, eps = 0.01), against the oracle's labels at every grid point
and against the plain evaluation of every point.  A point whose sigma lies within the parity
bar of eps may go either way; every other label must agree."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import golden, need_gpu, tol

pytestmark = pytest.mark.gpu


def _api():
    need_gpu()
    from paper_2605_04550_amd import api
    return api


def test_labels_match_oracle_on_the_paper_class():
    api = _api()
    import torch
    g = golden("paper_labels")
    w = W.paper_label_workload(3)
    grid, eps = w["grid"], w["eps"]
    for m, band in enumerate(w["mats"]):
        mat = api.BandedMatrix.from_band(band)
        r = api.label_grid(mat, grid, eps)
        torch.cuda.synchronize()
        lab = r["label"].cpu().numpy().ravel()
        sig = r["sigma"].cpu().numpy().ravel()
        evals = int(r["evals"].item())
        s_or, l_or = g["sigma%d" % m], g["label%d" % m]
        bar = tol(band.fro, s_or)
        sure = np.abs(s_or - eps) > 2 * bar
        assert np.array_equal(lab[sure], l_or[sure]), (m, np.flatnonzero(lab[sure] != l_or[sure])[:10])
        done = sig >= 0
        assert np.all(np.abs(sig[done] - s_or[done]) <= bar[done])
        assert np.all(done[l_or == 1] | ~sure[l_or == 1])      # sensitive points are evaluated
        print("paper-class matrix %d: %d sensitive, %d of %d shifts evaluated (%.1f %%)"
              % (m, int(lab.sum()), evals, grid.npts, 100.0 * evals / grid.npts), flush=True)
        assert evals == int(done.sum()) and evals < 0.5 * grid.npts
        # the plain method on every point gives the same labels
        full = api.eval_grid(mat, grid, eps=eps)
        plain = full["sens"].cpu().numpy()
        assert np.array_equal(lab[sure], plain[sure])


def test_labels_edge_cases():
    api = _api()
    import torch
    band = W.paper_training_matrix(W.SEED_BASE + 6100)
    mat = api.BandedMatrix.from_band(band)
    z_all = None
    for grid, eps in [(W.Grid(-4.0, 4.0, -4.0, 4.0, 7, 5), 0.01),      # tiny grid: stride 1 only
                      (W.Grid(-4.0, 4.0, 0.5, 0.5, 61, 1), 0.05),      # one row
                      (W.Grid(0.3, 0.3, -4.0, 4.0, 1, 53), 0.05),      # one column
                      (W.Grid(-4.0, 4.0, -4.0, 4.0, 40, 40), 100.0),   # everything sensitive
                      (W.Grid(-4.0, 4.0, -4.0, 4.0, 40, 40), 1e-12)]:  # almost nothing sensitive
        r = api.label_grid(mat, grid, eps)
        full = api.eval_grid(mat, grid, eps=eps)
        lab = r["label"].cpu().numpy().ravel()
        s = full["sigma"].cpu().numpy()
        sure = np.abs(s - eps) > 2 * tol(band.fro, s)
        assert np.array_equal(lab[sure], full["sens"].cpu().numpy()[sure]), (grid, eps)
        ev = int(r["evals"].item())
        assert 1 <= ev <= grid.npts
        if eps == 100.0:
            assert lab.all() and ev == grid.npts        # no exclusion possible


def test_labels_with_capped_evaluations():
    """Labels when evaluations stop at a low iteration cap (Golub-Kahan only, max_iter = 2): on
    the Toeplitz (0.25, 0, 1) matrix outside the symbol curve the process needs hundreds of
    steps, so many points end with PS_PT_MAXITER and an estimate above eps.  Those points are
    reported as undecided (2) and size no exclusion disk: every 1 and every 0 still agrees with
    the plain method at the default cap (away from sigma = eps within the tolerance), for one
    matrix and for a batch."""
    api = _api()
    import torch
    band = W.toeplitz(400, 0.25, 0.0, 1.0)
    grid = W.Grid(-2.0, 2.0, -2.0, 2.0, 64, 64)
    eps = 1e-2
    mat = api.BandedMatrix.from_band(band)
    full = api.eval_grid(mat, grid, eps=eps)
    s = full["sigma"].cpu().numpy()
    assert np.all((full["info"].cpu().numpy() & 2) == 0)
    sure = np.abs(s - eps) > 2 * tol(band.fro, s)
    ref = full["sens"].cpu().numpy()
    r = api.label_grid(mat, grid, eps, max_iter=2, bisect=False)
    lab = r["label"].cpu().numpy().ravel()
    und = lab == 2
    print("capped labels: %d undecided of %d" % (und.sum(), lab.size), flush=True)
    assert und.sum() > 0 and set(np.unique(lab)) <= {0, 1, 2}
    dec = ~und & sure
    assert np.array_equal(lab[dec], ref[dec])
    # batch: the same matrix twice, plus a normal matrix whose labels are known exactly
    b2 = W.diagonal(np.linspace(-1, 1, 50) + 0.3j)
    g2 = W.Grid(-1.5, 1.5, -1.0, 1.0, 33, 21)
    mats = [api.BandedMatrix.from_band(b) for b in (band, band, b2)]
    batch = api.BandedBatch(mats, [grid, grid, g2])
    rb = batch.label(eps, max_iter=2, bisect=False)
    lb = rb["label"].cpu().numpy()
    for m in range(2):
        lm = lb[rb["offsets"][m]:rb["offsets"][m] + grid.npts]
        assert np.array_equal(lm == 2, und)
        assert np.array_equal(lm[dec], ref[dec])
    l3 = lb[rb["offsets"][2]:rb["offsets"][2] + g2.npts]
    z3 = oracle.grid_points(g2)
    d3 = np.min(np.abs(z3[:, None] - (np.linspace(-1, 1, 50) + 0.3j)[None]), axis=1)   # normal: exact
    dec3 = (l3 != 2) & (np.abs(d3 - eps) > 2 * tol(b2.fro, d3))
    print("capped labels, normal matrix: %d decided of %d" % (dec3.sum(), l3.size), flush=True)
    assert dec3.any() and np.array_equal(l3[dec3] == 1, (d3 <= eps)[dec3])


def test_batched_labels_match_single_matrix_and_oracle():
    """ps_label_batch over matrices of the label workload (plus one matrix on a small ragged
    grid of its own): per matrix the labels of ps_label_grid and, for the three with stored
    oracle values, the oracle's labels."""
    api = _api()
    import torch
    g = golden("paper_labels")
    w = W.paper_label_workload(8)
    grid, eps = w["grid"], w["eps"]
    bands = list(w["mats"]) + [W.paper_training_matrix(W.SEED_BASE + 6200)]
    grids = [grid] * 8 + [W.Grid(-3.0, 2.0, -1.0, 4.0, 37, 29)]
    mats = [api.BandedMatrix.from_band(b) for b in bands]
    batch = api.BandedBatch(mats, grids)
    r = batch.label(eps)
    torch.cuda.synchronize()
    lab = r["label"].cpu().numpy()
    sig = r["sigma"].cpu().numpy()
    total_evals = 0
    for m, (band, gr) in enumerate(zip(bands, grids)):
        off = r["offsets"][m]
        lm = lab[off:off + gr.npts]
        sm = sig[off:off + gr.npts]
        single = api.label_grid(mats[m], gr, eps)
        ls = single["label"].cpu().numpy().ravel()
        full = api.eval_grid(mats[m], gr, eps=eps)
        sf = full["sigma"].cpu().numpy()
        sure = np.abs(sf - eps) > 2 * tol(band.fro, sf)
        assert np.array_equal(lm[sure], ls[sure]) and np.array_equal(lm[sure], full["sens"].cpu().numpy()[sure]), m
        done = sm >= 0
        assert np.all(np.abs(sm[done] - sf[done]) <= tol(band.fro, sf[done]))
        total_evals += int(done.sum())
        if m < 3:
            s_or, l_or = g["sigma%d" % m], g["label%d" % m]
            sure_o = np.abs(s_or - eps) > 2 * tol(band.fro, s_or)
            assert np.array_equal(lm[sure_o], l_or[sure_o]), m
    assert int(r["evals"].item()) == total_evals
    npts = sum(gr.npts for gr in grids)
    print("batched labels: %d matrices, %d of %d shifts evaluated (%.1f %%)"
          % (len(bands), total_evals, npts, 100.0 * total_evals / npts), flush=True)


def test_label_batch_at_the_benchmarked_size():
    """The launch the label benchmark times: all 500 matrices of the workload in one
    ps_label_batch.  Every label equals the plain method's (sigma_min <= eps from ps_eval_batch on
    every point) wherever sigma is further than twice the tolerance from eps, and the first
    three matrices match the oracle's stored labels."""
    api = _api()
    import torch
    g = golden("paper_labels")
    w = W.paper_label_workload(500)
    grid, eps = w["grid"], w["eps"]
    mats = [api.BandedMatrix.from_band(b) for b in w["mats"]]
    batch = api.BandedBatch(mats, [grid] * len(mats))
    r = batch.label(eps)
    p = batch.eval(None)
    torch.cuda.synchronize()
    lab = r["label"].cpu().numpy()
    sp = p["sigma"].cpu().numpy()
    fro = np.repeat([b.fro for b in w["mats"]], grid.npts)
    sure = np.abs(sp - eps) > 2 * tol(fro, sp)
    assert np.array_equal(lab[sure], (sp[sure] <= eps).astype(np.uint8))
    for m in range(3):
        off = r["offsets"][m]
        s_or, l_or = g["sigma%d" % m], g["label%d" % m]
        sure_o = np.abs(s_or - eps) > 2 * tol(w["mats"][m].fro, s_or)
        assert np.array_equal(lab[off:off + grid.npts][sure_o], l_or[sure_o]), m
    print("label batch of 500: %d of %d labels decided away from eps, %d evaluations"
          % (int(sure.sum()), len(sp), int(r["evals"].item())), flush=True)
