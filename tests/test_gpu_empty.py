"""GPU tests of the degenerate inputs of the C ABI: no shifts at all (a call with npts = 0, a
mask with no point set, a matrix of a batch whose mask is empty, the adjoint of no points) and
the 1 x 1 matrix, whose smallest singular value at z is |z - a| exactly."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import need_gpu, tol

pytestmark = pytest.mark.gpu


def test_no_shifts():
    torch = need_gpu()
    import paper_2605_04550_amd as P
    from paper_2605_04550_amd import api
    band = W.random_banded(50, 1, 2, seed=61)
    mat = api.BandedMatrix.from_band(band)
    # npts = 0 through the C ABI: accepted, nothing written (the outputs keep their sentinels)
    z = torch.zeros(1, dtype=torch.complex128, device="cuda")
    sig = torch.full((1,), -7.0, dtype=torch.float64, device="cuda")
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    for vec in (False, True):
        o = api.make_opts(want_vectors=vec)
        ws = torch.empty(max(1, P.ps_workspace_size(mat.handle, 0, o)), dtype=torch.uint8, device="cuda")
        u = torch.full((1, band.n), -7.0, dtype=torch.complex128, device="cuda")
        P.ps_eval_points(mat.handle, z.data_ptr(), 0, o, ws.data_ptr(), ws.numel(), sig.data_ptr(),
                         u.data_ptr() if vec else 0, u.data_ptr() if vec else 0, info.data_ptr(), 0, 0)
        torch.cuda.synchronize()
        assert sig.item() == -7.0 and info.item() == -7
        assert bool((u == -7.0).all())
    # a grid whose mask sets no point
    g = W.Grid(-2.0, 2.0, -2.0, 2.0, 17, 9)
    empty = torch.zeros((g.ny, g.nx), dtype=torch.uint8, device="cuda")
    for vec in (False, True):
        r = api.eval_grid(mat, g, empty, want_vectors=vec)
        torch.cuda.synchronize()
        assert int(r["count"].item()) == 0
    # the adjoint of no points: the band gradient is all zeros (it is overwritten)
    gs = torch.empty(0, dtype=torch.float64, device="cuda")
    uv = torch.empty((0, band.n), dtype=torch.complex128, device="cuda")
    gz, gb = api.backward(mat, gs, uv, uv)
    torch.cuda.synchronize()
    assert gz.numel() == 0 and bool((gb == 0).all())


def test_batch_with_an_empty_mask():
    torch = need_gpu()
    from paper_2605_04550_amd import api
    bands = [W.random_banded(80, 1, 1, seed=62), W.random_banded(60, 2, 1, seed=63), W.random_banded(70, 0, 2, seed=64)]
    grids = [W.Grid(*W.gershgorin_box(b), 9, 7) for b in bands]
    mats = [api.BandedMatrix.from_band(b) for b in bands]
    batch = api.BandedBatch(mats, grids)
    masks = [torch.zeros((g.ny, g.nx), dtype=torch.uint8, device="cuda") for g in grids]
    masks[1][::2, ::3] = 1                      # one matrix with points, the others none
    r = batch.eval(masks)
    torch.cuda.synchronize()
    counts = r["counts"].cpu().numpy()
    want = int(masks[1].sum().item())
    assert counts.tolist() == [0, want, 0]
    off = r["offsets"][1]
    idx = r["idx"][off:off + want].cpu().numpy()
    assert np.array_equal(idx, oracle.compact_mask(masks[1].cpu().numpy()))
    z = oracle.grid_points(grids[1])[idx]
    ref = oracle.sigma_min(bands[1], z)["sigma"]
    sb = r["sigma"][off:off + want].cpu().numpy()
    assert np.all(np.abs(sb - ref) <= tol(bands[1].fro, ref))
    # every mask empty: nothing to do, all counts zero
    r0 = batch.eval([torch.zeros_like(m) for m in masks])
    torch.cuda.synchronize()
    assert r0["counts"].cpu().numpy().tolist() == [0, 0, 0]


def test_one_by_one_matrix():
    torch = need_gpu()
    from paper_2605_04550_amd import api
    a = 0.3 - 1.7j
    band = W.diagonal([a])
    mat = api.BandedMatrix.from_band(band)
    rng = np.random.default_rng(65)
    z = np.concatenate([[a, a + 1e-9, a + 3.0j], rng.uniform(-3, 3, 13) + 1j * rng.uniform(-3, 3, 13)])
    zt = torch.tensor(z, dtype=torch.complex128, device="cuda")
    exact = np.abs(z - a)                       # sigma_min of the 1 x 1 matrix z - a
    for vec in (False, True):
        r = api.sigma_min(mat, zt, want_vectors=vec)
        s = r["sigma"].cpu().numpy()
        assert np.all(np.abs(s - exact) <= tol(band.fro, exact)), (vec, s, exact)
        if vec:
            # the pair of every nonsingular shift (z = a itself is reported singular, sigma 0)
            nz = exact > 0
            u, v = r["u"].cpu().numpy()[nz, 0], r["v"].cpu().numpy()[nz, 0]
            assert np.allclose(np.abs(u), 1.0) and np.allclose(np.abs(v), 1.0)
            # (z - a) v = sigma u
            assert np.allclose((z[nz] - a) * v, s[nz] * u, atol=1e-14)
    info = api.sigma_min(mat, zt)["info"].cpu().numpy()
    assert info[0] & 1 and not np.any(info[1:] & 1)   # PS_PT_SINGULAR at z = a only
