"""GPU tests of matrices wider than the banded kernels (kl or ku > 4, n <= 64), which take the
dense sigma-only path: the paper's Jordan example of Sec. 2 and seeded wide-band and full
matrices against the oracle, through ps_eval_points and ps_eval_grid (full and masked), and the
entry points that refuse such matrices."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import need_gpu, tol

pytestmark = pytest.mark.gpu


def _api():
    need_gpu()
    from paper_2605_04550_amd import api
    return api


def _read_jordan():
    import os
    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "jordan32.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_jordan_example_of_sec2():
    """Sec. 2: sigma_min(0 I - J) = 0 for the 32 x 32 Jordan block J; B = J + 0.01 in the first row,
    last column (kl = 1, ku = 31) has its 32 eigenvalues on the circle of radius 0.01^(1/32), where
    sigma_min(lambda I - B) = 0; off the circle sigma_min(zI - B) > 0 meets the oracle's value."""
    api = _api()
    import torch
    g = _read_jordan()
    J = W.jordan(32)
    B = W.jordan_perturbed(32, g["delta"])
    mj = api.BandedMatrix.from_band(J)
    mb = api.BandedMatrix.from_band(B)
    print("Jordan example: B has kl = %d, ku = %d (dense path)" % (B.kl, B.ku), flush=True)
    s0 = api.sigma_min(mj, torch.tensor([0.0 + 0.0j], dtype=torch.complex128, device="cuda"))["sigma"].item()
    assert s0 <= tol(J.fro, 0.0)
    lam = g["eigenvalue_modulus"] * np.exp(2j * np.pi * np.arange(32) / 32)
    r = api.sigma_min(mb, torch.tensor(lam, dtype=torch.complex128, device="cuda"))
    sb = r["sigma"].cpu().numpy()
    print("Jordan example: max sigma_min at B's eigenvalues %.3e (bar %.3e)" % (sb.max(), tol(B.fro, 0.0)),
          flush=True)
    assert np.all(sb <= tol(B.fro, 0.0))
    assert np.all(r["info"].cpu().numpy() == 0)
    zoff = np.array([0.0, 0.5 + 0.5j, 1.2, -0.9j, 0.3 - 0.2j])
    so = api.sigma_min(mb, torch.tensor(zoff, dtype=torch.complex128, device="cuda"))["sigma"].cpu().numpy()
    ref = oracle.sigma_min(B, zoff)["sigma"]
    assert np.all(np.abs(so - ref) <= tol(B.fro, ref))


@pytest.mark.parametrize("n,kl,ku", [(7, 6, 0), (12, 5, 5), (17, 2, 9), (40, 11, 7), (64, 63, 63), (64, 5, 1)])
def test_wide_bands_against_oracle(n, kl, ku):
    """Seeded complex matrices with kl or ku > 4 (up to a full 64 x 64): sigma at a list of shifts
    and on a 9 x 7 grid, full and masked, within the bar of the oracle's dense Jacobi SVD."""
    api = _api()
    import torch
    band = W.random_banded(n, kl, ku, seed=1000 + 10 * n + kl + ku)
    mat = api.BandedMatrix.from_band(band)
    rng = np.random.default_rng(77 + n)
    z = 2.0 * (rng.standard_normal(24) + 1j * rng.standard_normal(24))
    r = api.sigma_min(mat, torch.tensor(z, dtype=torch.complex128, device="cuda"))
    got = r["sigma"].cpu().numpy()
    ref = oracle.sigma_min(band, z)["sigma"]
    err = np.abs(got - ref) / tol(band.fro, ref)
    print("n=%d kl=%d ku=%d: list max err/bound %.3e" % (n, kl, ku, err.max()), flush=True)
    assert np.all(err <= 1.0)
    grid = W.Grid(-3.0, 2.5, -2.0, 3.0, 9, 7)
    zg = oracle.grid_points(grid)
    refg = oracle.sigma_min(band, zg)["sigma"]
    full = api.eval_grid(mat, grid, eps=0.5)
    cnt = int(full["count"].item())
    assert cnt == grid.npts
    assert np.array_equal(full["idx"][:cnt].cpu().numpy(), np.arange(grid.npts))
    sg = full["sigma"][:cnt].cpu().numpy()
    assert np.all(np.abs(sg - refg) <= tol(band.fro, refg))
    assert np.array_equal(full["sens"][:cnt].cpu().numpy(), oracle.sensitive(sg, 0.5))
    mask = (rng.uniform(size=(grid.ny, grid.nx)) < 0.4).astype(np.uint8)
    mr = api.eval_grid(mat, grid, torch.tensor(mask, device="cuda"))
    cm = int(mr["count"].item())
    idx = oracle.compact_mask(mask)
    assert cm == len(idx) and np.array_equal(mr["idx"][:cm].cpu().numpy(), idx)
    sm = mr["sigma"][:cm].cpu().numpy()
    assert np.all(np.abs(sm - refg[idx]) <= tol(band.fro, refg[idx]))


def test_wide_band_refusals():
    """Entry points that need the banded kernels refuse a dense-path matrix with
    PS_ERR_UNSUPPORTED: vectors, batches, labels, the allocation-free call, the adjoint."""
    api = _api()
    import torch
    import paper_2605_04550_amd as P
    band = W.random_banded(20, 6, 2, seed=5)
    mat = api.BandedMatrix.from_band(band)
    z = torch.tensor([0.1 + 0.2j, 1.0], dtype=torch.complex128, device="cuda")
    with pytest.raises(P.PsError) as e:
        api.sigma_min(mat, z, want_vectors=True)
    assert e.value.status == P.PS_ERR_UNSUPPORTED
    with pytest.raises(P.PsError) as e:
        api.BandedBatch([mat], [W.Grid(-1, 1, -1, 1, 4, 4)])
    assert e.value.status == P.PS_ERR_UNSUPPORTED
    with pytest.raises(P.PsError) as e:
        api.label_grid(mat, W.Grid(-1, 1, -1, 1, 4, 4), 0.1)
    assert e.value.status == P.PS_ERR_UNSUPPORTED
    sig = torch.empty(2, dtype=torch.float64, device="cuda")
    with pytest.raises(P.PsError) as e:
        P.ps_eval_points_noalloc(mat.handle, z.data_ptr(), 2, None, sig.data_ptr(), 0, 0, 0)
    assert e.value.status == P.PS_ERR_UNSUPPORTED
    u = torch.zeros((2, 20), dtype=torch.complex128, device="cuda")
    with pytest.raises(P.PsError) as e:
        api.backward(mat, torch.ones(2, dtype=torch.float64, device="cuda"), u, u)
    assert e.value.status == P.PS_ERR_UNSUPPORTED
