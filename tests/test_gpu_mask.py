"""GPU parity of the mask producer (ps_mlp_prob, ps_mask_predict) against the oracle
(``oracle/mask.py``): the classifier of Sec. 3.2 and the hierarchical prediction of Sec. 3.5.

Probabilities: |p_gpu - p_oracle| within the oracle's first-order bound for a float32
evaluation, per point.  Decisions (the coarse percentile, the refined cells, p >= tau, the
dilation): the oracle's rule is fed the GPU's own float32 probabilities, and the GPU's
tau_coarse, refined cells, probability map, mask and evaluation count must then be identical.
Weights, global features and spectra are seeded draws (``workloads.nets``); the paper's
trained weights are not available."""
import numpy as np
import pytest

import workloads as W
from gpu_util import need_gpu
from oracle import mask as OM
from workloads import nets

pytestmark = pytest.mark.gpu


def _api():
    need_gpu()
    from paper_2605_04550_amd import api
    return api


def _t(x, dtype):
    import torch
    return torch.tensor(x, dtype=dtype, device="cuda")


def _check_prob(p_gpu, params, gf, eig, z, what):
    p_or, e = OM.mlp_prob(params, gf, eig, z, bound=True)
    err = np.abs(p_gpu.astype(np.float64) - p_or)
    worst = int(np.argmax(err / e))
    print("%s: %d points, max |dp| %.2e, max |dp| / bound %.3f (p std %.3f)"
          % (what, len(z), err.max(), (err / e)[worst], p_or.std()), flush=True)
    assert np.all(err <= e + 1e-30), (what, worst, p_gpu[worst], p_or[worst], e[worst])
    return p_or, e


@pytest.mark.parametrize("scale,neig,npts", [(1.0, 64, 1000), (3.0, 23, 517), (3.0, 1, 37), (2.0, 301, 16)])
def test_mlp_prob_vs_oracle(scale, neig, npts):
    api = _api()
    import torch
    params = nets.mlp_params(11, scale)
    gf = nets.global_features(12)
    eig = nets.spectrum(13, neig)
    rng = np.random.default_rng(14)
    z = rng.uniform(-4, 4, npts) + 1j * rng.uniform(-4, 4, npts)
    net = api.MaskNet(params)
    p = net.prob(gf, _t(eig, torch.complex128), _t(z, torch.complex128))
    torch.cuda.synchronize()
    _check_prob(p.cpu().numpy(), params, gf, eig, z, "prob scale %g neig %d" % (scale, neig))
    # a device-resident parameter vector gives the same network
    net2 = api.MaskNet(_t(params, torch.float32))
    p2 = net2.prob(gf, _t(eig, torch.complex128), _t(z, torch.complex128))
    assert torch.equal(p, p2)
    # no points: nothing to do
    assert net.prob(gf, _t(eig, torch.complex128), _t(np.zeros(0), torch.complex128)).numel() == 0


def _run_mask(api, grid, params, gf, eig, tau, stride, dilate, q=0.8):
    import torch
    net = api.MaskNet(params)
    r = net.predict(grid, gf, _t(eig, torch.complex128), tau=tau, stride=stride, dilate=dilate, coarse_q=q)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items()}


def _check_mask(grid, params, gf, eig, tau, stride, dilate, r, q=0.8, what=""):
    cy, cx = OM.coarse_shape(grid, stride)
    assert r["coarse"].shape == (cy, cx) and r["prob"].shape == (grid.ny, grid.nx)
    # coarse probabilities vs the oracle
    ci, cj = np.meshgrid(np.arange(cy), np.arange(cx), indexing="ij")
    cflat = (stride * ci * grid.nx + stride * cj).ravel()
    _check_prob(r["coarse"].ravel(), params, gf, eig, OM.mask_points_z(grid, cflat), what + " coarse")
    # the oracle's rule on the GPU's own probabilities: identical decisions
    gprob = r["prob"].astype(np.float64).ravel()
    ref = OM.hierarchical_mask(grid, lambda flat: gprob[np.asarray(flat)], tau, stride=stride, q=q, dilate=dilate,
                               coarse=r["coarse"].astype(np.float64))
    assert float(r["tau_coarse"]) == ref["tau_coarse"], (float(r["tau_coarse"]), ref["tau_coarse"])
    np.testing.assert_array_equal(r["prob"].astype(np.float64), ref["prob"])     # zeros exactly off the refined cells
    np.testing.assert_array_equal(r["mask"], ref["mask"])
    assert int(r["evals"][0]) == ref["evals"]
    # fine probabilities of the refined cells vs the oracle
    fine = np.flatnonzero(np.kron(ref["selected"], np.ones((stride, stride), dtype=bool))[:grid.ny, :grid.nx].ravel())
    if fine.size:
        _check_prob(r["prob"].ravel()[fine], params, gf, eig, OM.mask_points_z(grid, fine), what + " fine")
    return ref


def test_mask_predict_paper_grid_vs_oracle():
    """The Sec. 3.5 setting: 100 x 100 grid on [-4, 4]^2, stride 4 (625 coarse points), 80th
    percentile, 5 x 5 dilation; a 64-point spectrum."""
    api = _api()
    grid = W.Grid(-4.0, 4.0, -4.0, 4.0, 100, 100)
    params, gf, eig = nets.mlp_params(21, 3.0), nets.global_features(22), nets.spectrum(23, 64)
    for tau in (0.05, 0.3, 0.6):
        r = _run_mask(api, grid, params, gf, eig, tau, 4, 5)
        ref = _check_mask(grid, params, gf, eig, tau, 4, 5, r, what="paper grid tau %g" % tau)
        print("tau %g: tau_coarse %.4f, %d refined cells, %d evaluations, |R| = %d"
              % (tau, ref["tau_coarse"], ref["selected"].sum(), int(r["evals"][0]), int(r["mask"].sum())), flush=True)
        assert ref["selected"].sum() >= 125                    # at least the top 20 % of 625 cells
        # end to end against the float64 oracle: masks agree except where a decision sits
        # within the float32 error of its threshold
        full = OM.mask_predict(params, gf, eig, grid, tau)
        diff = np.flatnonzero(full["mask"].ravel() != r["mask"].ravel())
        if diff.size:
            pc, ec = OM.mlp_prob(params, gf, eig, OM.mask_points_z(grid, np.arange(grid.npts)), bound=True)
            near = np.abs(pc - tau) <= ec
            near_c = abs(full["tau_coarse"] - float(r["tau_coarse"])) > 0
            assert near.any() or near_c, diff[:10]
        print("  float64 oracle mask differs at %d points" % diff.size, flush=True)


@pytest.mark.parametrize("shape,stride,dilate,tau,neig", [
    ((37, 23), 4, 5, 0.4, 23), ((1, 1), 4, 5, 0.1, 1), ((13, 1), 4, 1, 0.5, 5), ((1, 30), 3, 5, 0.2, 7),
    ((50, 61), 8, 3, 0.6, 64), ((17, 9), 2, 7, 0.4, 64), ((100, 100), 1, 1, 0.5, 10), ((64, 64), 16, 31, 0.7, 3),
    ((33, 47), 5, 9, 1.0, 40)])
def test_mask_predict_ragged_and_edge_cases(shape, stride, dilate, tau, neig):
    api = _api()
    nx, ny = shape
    grid = W.Grid(-3.0, 2.5, -1.5, 4.0, nx, ny)
    params, gf, eig = nets.mlp_params(31 + nx, 3.0), nets.global_features(32), nets.spectrum(33 + ny, neig)
    r = _run_mask(api, grid, params, gf, eig, tau, stride, dilate)
    _check_mask(grid, params, gf, eig, tau, stride, dilate, r, what="%dx%d s%d d%d" % (nx, ny, stride, dilate))


def test_mask_feeds_the_restricted_evaluation():
    """Sec. 4: sigma_min only on R.  The predicted mask goes straight into ps_eval_grid; the
    values on R equal the full-grid values at the same points (same arithmetic)."""
    api = _api()
    import torch
    band = W.paper_training_matrix(W.SEED_BASE + 6000)
    A = W.to_dense(band)
    eig = np.linalg.eigvals(A)                      # input preparation: the spectrum of A
    grid = W.Grid(-4.0, 4.0, -4.0, 4.0, 100, 100)
    params, gf = nets.mlp_params(41, 3.0), nets.global_features(42)
    net = api.MaskNet(params)
    r = net.predict(grid, gf, _t(eig, torch.complex128), tau=0.3)
    mat = api.BandedMatrix.from_band(band)
    full = api.eval_grid(mat, grid, eps=0.01)
    res = api.eval_grid(mat, grid, r["mask"], eps=0.01)
    torch.cuda.synchronize()
    c = int(res["count"].item())
    idx = res["idx"][:c].cpu().numpy()
    np.testing.assert_array_equal(idx, np.flatnonzero(r["mask"].cpu().numpy().ravel()))
    np.testing.assert_allclose(res["sigma"][:c].cpu().numpy(), full["sigma"].cpu().numpy()[idx], rtol=1e-13, atol=0)
    print("restricted evaluation: |R| = %d of %d points" % (c, grid.npts), flush=True)


@pytest.mark.parametrize("shape,stride,dilate,tau", [((37, 23), 4, 5, 0.4), ((100, 100), 4, 5, 0.05),
                                                     ((33, 47), 5, 9, 0.5)])
def test_mask_predict_batch_equals_single_calls(shape, stride, dilate, tau):
    """ps_mask_predict_batch runs the single call's kernels with a matrix index: every output of
    every matrix is identical to the single call's; one matrix also against the oracle."""
    api = _api()
    import torch
    nx, ny = shape
    grid = W.Grid(-4.0, 4.0, -3.0, 3.5, nx, ny)
    sizes = [1, 5, 64, 64, 23, 300, 2]
    params = nets.mlp_params(51, 3.0)
    gfs = np.stack([nets.global_features(60 + m) for m in range(len(sizes))])
    eigs = [nets.spectrum(70 + m, n) for m, n in enumerate(sizes)]
    net = api.MaskNet(params)
    teigs = [_t(e, torch.complex128) for e in eigs]
    rb = net.predict_batch(grid, gfs, teigs, tau=tau, stride=stride, dilate=dilate)
    torch.cuda.synchronize()
    for m in range(len(sizes)):
        r1 = net.predict(grid, gfs[m], teigs[m], tau=tau, stride=stride, dilate=dilate)
        torch.cuda.synchronize()
        for k in ("mask", "prob", "coarse"):
            assert torch.equal(rb[k][m], r1[k]), (m, k)
        assert float(rb["tau_coarse"][m]) == float(r1["tau_coarse"]), m
        assert int(rb["evals"][m]) == int(r1["evals"][0]), m
    r = {k: v[4].cpu().numpy() for k, v in rb.items()}
    r["evals"] = np.array([r["evals"]])
    _check_mask(grid, params, gfs[4], eigs[4], tau, stride, dilate, r, what="batch matrix 4")


def _check_calibration(api, grid, prob, labels, taus, **kw):
    import torch
    r = api.calibrate_tau(grid, _t(prob, torch.float32), _t(labels, torch.uint8), taus, **kw)
    torch.cuda.synchronize()
    o = OM.calibrate_tau(prob.astype(np.float32).astype(np.float64), labels, taus,
                         **{k: v for k, v in kw.items()})
    np.testing.assert_array_equal(r["recall"].cpu().numpy(), o["recall"])
    np.testing.assert_array_equal(r["median"].cpu().numpy(), o["median"])
    np.testing.assert_array_equal(r["p10"].cpu().numpy(), o["p10"])
    assert (r["index"], r["index_max"]) == (o["index"], o["index_max"])
    return r


def test_calibration_vs_oracle():
    """ps_mask_calibrate against the oracle on the same maps: recalls (ratios of counts), their
    median and 10th percentile, and both qualifying indices, all identical."""
    api = _api()
    rng = np.random.default_rng(17)
    nval, ny, nx = 9, 23, 31
    grid = W.Grid(0.0, 1.0, 0.0, 1.0, nx, ny)
    prob = (rng.uniform(size=(nval, ny, nx)) ** 13).astype(np.float32)
    labels = (rng.uniform(size=(nval, ny, nx)) < 0.03).astype(np.uint8)
    labels[4] = 0
    taus = [round(0.05 + 0.01 * k, 2) for k in range(90)]
    r = _check_calibration(api, grid, prob, labels, taus)
    assert r["index"] == 0 and 0 < r["index_max"] < 89
    # other dilations and bounds; no candidate qualifies; a single matrix and candidate
    _check_calibration(api, grid, prob, labels, taus, pred_dilate=3, label_dilate=1, median_min=0.8, p10_min=0.5)
    r = _check_calibration(api, grid, prob, labels, taus, median_min=1.01)
    assert (r["index"], r["index_max"]) == (-1, -1)
    _check_calibration(api, grid, prob[:1], labels[:1], [0.3])
    r = _check_calibration(api, grid, prob, np.zeros_like(labels), taus)
    assert (r["index"], r["index_max"]) == (0, 89)


def test_calibration_on_predicted_maps_and_exact_labels():
    """The Sec. 3.6 procedure end to end on the GPU: 30 validation matrices of the Sec. 3.3 class,
    probability maps from ps_mask_predict_batch, labels from ps_label_batch (exact, eps = 0.01);
    the oracle's calibration on the same two arrays gives the same answer."""
    api = _api()
    import torch
    w = W.paper_label_workload(30)
    grid = w["grid"]
    mats = [api.BandedMatrix.from_band(b) for b in w["mats"]]
    batch = api.BandedBatch(mats, [grid] * len(mats))
    lab = batch.label(w["eps"])["label"].reshape(30, grid.ny, grid.nx)
    net = api.MaskNet(nets.mlp_params(91, 3.0))
    eigs = [_t(np.linalg.eigvals(W.to_dense(b)), torch.complex128) for b in w["mats"]]
    gfs = np.stack([nets.global_features(92 + m) for m in range(30)])
    pr = net.predict_batch(grid, gfs, eigs, tau=0.05)["prob"]
    torch.cuda.synchronize()
    taus = [round(0.05 + 0.01 * k, 2) for k in range(90)]
    r = _check_calibration(api, grid, pr.cpu().numpy(), lab.cpu().numpy(), taus)
    print("calibration on 30 matrices: tau* index %d, largest qualifying %d, median recall at 0.05 %.3f"
          % (r["index"], r["index_max"], float(r["median"][0])), flush=True)


def test_mask_batch_at_the_benchmarked_size():
    """The launch the mask benchmark times: 500 matrices of the Sec. 3.3 class, the 100 x 100
    grid, the same weights and features.  Sampled matrices equal their single calls exactly,
    and one of them matches the oracle (probabilities within the bound, decisions identical)."""
    api = _api()
    import torch
    w = W.paper_label_workload(500)
    grid = w["grid"]
    params = nets.mlp_params(W.SEED_BASE + 900, 3.0)
    net = api.MaskNet(params)
    eig_np = [np.linalg.eigvals(W.to_dense(b)) for b in w["mats"]]
    eigs = [_t(e, torch.complex128) for e in eig_np]
    gfs = np.stack([nets.global_features(W.SEED_BASE + 901 + m) for m in range(500)])
    rb = net.predict_batch(grid, gfs, eigs, tau=0.05)
    torch.cuda.synchronize()
    assert int(rb["evals"].min()) >= 2625
    for m in (0, 137, 311, 499):
        r1 = net.predict(grid, gfs[m], eigs[m], tau=0.05)
        torch.cuda.synchronize()
        for k in ("mask", "prob", "coarse"):
            assert torch.equal(rb[k][m], r1[k]), (m, k)
    r = {k: v[311].cpu().numpy() for k, v in rb.items()}
    r["evals"] = np.array([r["evals"]])
    _check_mask(grid, params, gfs[311], eig_np[311], 0.05, 4, 5, r, what="benchmarked batch, matrix 311")


def test_trained_network_on_held_out_matrices():
    """The trained classifier (paper_2605_04550_amd/data/mask_net.npz, written by the training
    script): ps_mlp_prob equals the oracle's float64 network within its float32 error bound on the
    real features of a held-out matrix (plus float32 underflow); on 20 held-out matrices of the Sec. 3.3 class the region R
    at the calibrated tau* (hierarchical prediction, 5 x 5 dilation) covers the exact labels
    (dilated 3 x 3, as in the calibration of Sec. 3.6) with median recall >= 0.90 and 10th
    percentile >= 0.75, the bounds tau* was calibrated to."""
    need_gpu()
    import os
    import scipy.ndimage as nd
    import torch
    from paper_2605_04550_amd import api
    from paper_2605_04550_amd.features import band_features
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2605_04550_amd", "data",
                        "mask_net.npz")
    if not os.path.exists(path):
        pytest.skip("no trained weights")
    tw = np.load(path, allow_pickle=False)
    params, tau = tw["params"], float(tw["tau"])
    net = api.MaskNet(params)
    w = W.paper_label_workload(20)
    grid = w["grid"]
    fe = [band_features(b, 3_000_000 + m) for m, b in enumerate(w["mats"])]
    rng = np.random.default_rng(41)
    z = rng.uniform(-4, 4, 512) + 1j * rng.uniform(-4, 4, 512)
    eig0 = torch.tensor(fe[0][1], dtype=torch.complex128, device="cuda")
    p = net.prob(list(fe[0][0]), eig0, torch.tensor(z, dtype=torch.complex128, device="cuda")).double().cpu().numpy()
    ref, bnd = OM.mlp_prob(params, fe[0][0], fe[0][1], z, bound=True)
    # the trained logits reach -90 far from the spectrum: probabilities below float32's normal
    # range (2^-126) may be flushed to zero, which the rounding bound does not model
    assert np.all(np.abs(p - ref) <= bnd + 2.0 ** -126)
    eigs = [torch.tensor(lam, dtype=torch.complex128, device="cuda") for _, lam in fe]
    rs = net.predict_batch(grid, [list(f) for f, _ in fe], eigs, tau=tau)
    mats = [api.BandedMatrix.from_band(b) for b in w["mats"]]
    lab = api.BandedBatch(mats, [grid] * len(mats)).label(w["eps"])["label"].reshape(20, grid.ny, grid.nx)
    lab = lab.cpu().numpy().astype(bool)
    rmask = rs["mask"].cpu().numpy().astype(bool)
    rec = []
    for m in range(20):
        dl = nd.binary_dilation(lab[m], structure=np.ones((3, 3), dtype=bool))
        rec.append(1.0 if dl.sum() == 0 else float((dl & rmask[m]).sum()) / float(dl.sum()))
    print("trained network, tau* %.2f: recall median %.3f, P10 %.3f, region fraction %.3f"
          % (tau, np.median(rec), np.percentile(rec, 10), rmask.mean()), flush=True)
    assert np.median(rec) >= 0.90 and np.percentile(rec, 10) >= 0.75
    assert rmask.mean() < 0.5
