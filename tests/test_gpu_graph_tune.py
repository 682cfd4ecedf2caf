"""GPU tests: the eval calls captured in a HIP graph (replayed several times with eager work
in between, each replay checked against the eager result), and the autotuner."""
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


def test_graph_capture_replays_match_eager():
    api = _api()
    import torch
    w = W.workload("grcar100")
    mat = api.BandedMatrix.from_band(w["band"])
    grid = w["grid"]
    rng = np.random.default_rng(3)
    mask = torch.tensor((rng.uniform(size=(grid.ny, grid.nx)) < 0.3).astype(np.uint8), device="cuda")
    eager_full = api.eval_grid(mat, grid, eps=1e-3)
    eager_mask = api.eval_grid(mat, grid, mask, eps=1e-3)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):          # warm-up on the capture stream
        api.eval_grid(mat, grid, eps=1e-3)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        full = api.eval_grid(mat, grid, eps=1e-3)
        masked = api.eval_grid(mat, grid, mask, eps=1e-3)
    for rep in range(3):
        full["sigma"].fill_(-1.0)
        masked["sigma"].fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        # some eager work between replays
        junk = api.eval_grid(mat, W.Grid(0.0, 1.0, 0.0, 1.0, 7, 5))
        torch.cuda.synchronize()
        for ref, got in ((eager_full, full), (eager_mask, masked)):
            c = int(ref["count"].item())
            assert int(got["count"].item()) == c
            assert torch.equal(got["idx"][:c], ref["idx"][:c])
            assert torch.equal(got["sigma"][:c], ref["sigma"][:c]), "replay %d differs" % rep
            assert torch.equal(got["sens"][:c], ref["sens"][:c])
    gold = golden("grcar100_all")
    sig = full["sigma"].cpu().numpy()
    assert np.all(np.abs(sig - gold["sigma"]) <= tol(w["band"].fro, gold["sigma"]))


def test_graph_capture_of_batch_and_newton():
    api = _api()
    import torch
    bands = [W.random_banded(90 + 20 * m, 1 + m % 3, 2 - m % 2, seed=70 + m) for m in range(4)]
    grids = [W.Grid(*W.gershgorin_box(b), 9, 11) for b in bands]
    mats = [api.BandedMatrix.from_band(b) for b in bands]
    batch = api.BandedBatch(mats, grids)
    eager = batch.eval(None)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.eval(None)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        got = batch.eval(None)
    for rep in range(3):
        got["sigma"].fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(got["sigma"], eager["sigma"]), rep
        assert torch.equal(got["counts"], eager["counts"])


def test_autotune_returns_a_valid_plan():
    api = _api()
    import torch
    w = W.workload("grcar100")
    mat = api.BandedMatrix.from_band(w["band"])
    z = torch.tensor(oracle.grid_points(w["grid"]), dtype=torch.complex128, device="cuda")
    o = api.autotune(mat, z)
    assert o.slots >= 256 and o.slots % 256 == 0 and o.check_shift in (3, 4, 5)
    assert o.bisect == 0
    r = api.sigma_min(mat, z, slots=o.slots, bisect=o.bisect == 0)
    gold = golden("grcar100_all")
    sig = r["sigma"].cpu().numpy()
    assert np.all(np.abs(sig - gold["sigma"]) <= tol(w["band"].fro, gold["sigma"]))
    print("autotuned plan: slots %d, check_shift %d" % (o.slots, o.check_shift))
    off = api.autotune(mat, z, bisect=False)
    assert off.bisect == -1


def test_graph_capture_of_mask_predict():
    """ps_mask_predict captured in a HIP graph (kernels only, no memset or copy): every replay,
    with eager work in between, equals the eager result."""
    api = _api()
    import torch
    from workloads import nets
    grid = W.Grid(-4.0, 4.0, -4.0, 4.0, 61, 47)
    net = api.MaskNet(nets.mlp_params(81, 3.0))
    gf = nets.global_features(82)
    eig = torch.tensor(nets.spectrum(83, 40), dtype=torch.complex128, device="cuda")
    eager = net.predict(grid, gf, eig, tau=0.4)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        net.predict(grid, gf, eig, tau=0.4)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        got = net.predict(grid, gf, eig, tau=0.4)
    for rep in range(3):
        got["mask"].fill_(7)
        got["prob"].fill_(-1.0)
        got["evals"].fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        net.predict(W.Grid(0.0, 1.0, 0.0, 1.0, 9, 5), gf, eig, tau=0.2)      # eager work between replays
        torch.cuda.synchronize()
        for k in ("mask", "prob", "coarse", "tau_coarse", "evals"):
            assert torch.equal(got[k], eager[k]), (rep, k)
