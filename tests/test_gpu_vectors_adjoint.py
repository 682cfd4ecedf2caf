"""GPU parity for singular vectors, the adjoint (ps_backward) and Newton contour refinement.

Vectors are unique only up to a joint phase, and only where sigma_min is simple; they are
compared through phase-invariant quantities (|u_gpu^H u_or|, u^H v, residuals) at points
whose oracle gap s_2 / s_1 is at least 1.05.  Gradients are compared with the oracle's
adjoint built from the oracle's own vectors, with central differences of sigma_min, and with
closed forms (n = 1, diagonal A)."""
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


def test_grcar400_vectors_vs_oracle():
    api = _api()
    import torch
    g = golden("grcar400_vec")
    band = W.grcar(400)
    A = W.to_dense(band)
    mat = api.BandedMatrix.from_band(band)
    z = torch.tensor(g["z"], dtype=torch.complex128, device="cuda")
    r = api.sigma_min(mat, z, want_vectors=True, tol_rel=1e-12, tol_norm=1e-14)
    sig = r["sigma"].cpu().numpy()
    b = tol(band.fro, g["sigma"])
    report("grcar400 vec sigma", sig, g["sigma"], b)
    assert np.all(np.abs(sig - g["sigma"]) <= b)
    u, v = r["u"].cpu().numpy(), r["v"].cpu().numpy()
    gap = g["s2"] / np.maximum(g["sigma"], 1e-300)
    sel = np.flatnonzero((gap >= 1.05) & (g["sigma"] > 1e-12))
    assert len(sel) >= 8
    for p in sel:
        M = g["z"][p] * np.eye(400) - A
        assert abs(np.linalg.norm(u[p]) - 1) < 1e-10 and abs(np.linalg.norm(v[p]) - 1) < 1e-10
        res = np.linalg.norm(M @ v[p] - sig[p] * u[p])
        assert res <= 1e-8 * np.linalg.norm(A) + 1e-6 * sig[p], (p, res)
        # sine of the angle to the oracle's vectors (phase-free)
        su = np.sqrt(max(0.0, 1 - abs(np.vdot(g["u"][p], u[p])) ** 2))
        sv = np.sqrt(max(0.0, 1 - abs(np.vdot(g["v"][p], v[p])) ** 2))
        assert su < 1e-6 and sv < 1e-6, (p, su, sv)
        assert abs(np.vdot(u[p], v[p]) - np.vdot(g["u"][p], g["v"][p])) < 1e-6, p
        k = int(np.argmax(np.abs(v[p])))
        assert abs(v[p][k].imag) < 1e-12 and v[p][k].real > 0


def test_adjoint_vs_oracle_adjoint():
    api = _api()
    import torch
    g = golden("grcar400_vec")
    band = W.grcar(400)
    mat = api.BandedMatrix.from_band(band)
    gap = g["s2"] / np.maximum(g["sigma"], 1e-300)
    sel = np.flatnonzero((gap >= 1.05) & (g["sigma"] > 1e-12))
    z = g["z"][sel]
    w = np.random.default_rng(5).standard_normal(len(sel))
    r = api.sigma_min(mat, torch.tensor(z, dtype=torch.complex128, device="cuda"), want_vectors=True,
                      tol_rel=1e-12, tol_norm=1e-14)
    gz, gb = api.backward(mat, torch.tensor(w, device="cuda"), r["u"], r["v"])
    gz_o, gb_o = oracle.adjoint(band, g["u"][sel], g["v"][sel], w)
    np.testing.assert_allclose(gz.cpu().numpy(), gz_o, atol=1e-6)
    # Grcar is real: the handle carries PS_REAL_A, so the band gradient is the real part
    assert mat.real
    gbn = gb.cpu().numpy()
    assert np.all(gbn.imag == 0)
    np.testing.assert_allclose(gbn.real, gb_o.real, atol=1e-6 * np.abs(w).sum())


def test_adjoint_closed_forms():
    api = _api()
    import torch
    # diagonal A: sigma = |z - a_k| at the nearest k; d/dz = (z - a_k)/|z - a_k|; dA_kk = -(same)
    rng = np.random.default_rng(3)
    vals = np.array([0.0, 3.0 + 1.0j, -2.0 + 0.5j, 1.0 - 2.0j])
    band = W.diagonal(vals)
    mat = api.BandedMatrix.from_band(band)
    z = vals[rng.integers(0, 4, 16)] + 0.3 * np.exp(2j * np.pi * rng.uniform(0, 1, 16))
    r = api.sigma_min(mat, torch.tensor(z, dtype=torch.complex128, device="cuda"), want_vectors=True)
    ones = torch.ones(16, dtype=torch.float64, device="cuda")
    gz, gb = api.backward(mat, ones, r["u"], r["v"])
    near = np.argmin(np.abs(z[:, None] - vals[None, :]), axis=1)
    expect = (z - vals[near]) / np.abs(z - vals[near])
    np.testing.assert_allclose(gz.cpu().numpy(), expect, atol=1e-9)
    gband = np.zeros(4, dtype=complex)
    for p in range(16):
        gband[near[p]] -= expect[p]
    np.testing.assert_allclose(gb.cpu().numpy()[:, 0], gband, atol=1e-8)


def test_adjoint_vs_finite_differences():
    api = _api()
    import torch
    band = W.grcar(60)
    band.real = False          # gradient w.r.t. complex band entries (no real projection)
    mat = api.BandedMatrix.from_band(band)
    z = np.array([0.3 + 1.9j, 2.2 - 0.7j, -0.8 + 2.5j, 1.5 + 0.2j])
    ro = oracle.sigma_min(band, z, all_sv=True)
    s_sorted = np.sort(ro["sall"], axis=1)
    assert np.all(s_sorted[:, 1] / s_sorted[:, 0] >= 1.05)
    tight = dict(tol_rel=1e-15, tol_norm=1e-17, max_iter=400)
    r = api.sigma_min(mat, torch.tensor(z, dtype=torch.complex128, device="cuda"), want_vectors=True, **tight)
    gz, gb = api.backward(mat, torch.ones(4, dtype=torch.float64, device="cuda"), r["u"], r["v"])
    h = 1e-6

    def sig(zz, bb=band):
        m = api.BandedMatrix.from_band(bb)
        return api.sigma_min(m, torch.tensor(zz, dtype=torch.complex128, device="cuda"), **tight)["sigma"].cpu().numpy()
    fd = ((sig(z + h) - sig(z - h)) + 1j * (sig(z + 1j * h) - sig(z - 1j * h))) / (2 * h)
    np.testing.assert_allclose(gz.cpu().numpy(), fd, atol=2e-6)
    gbn = gb.cpu().numpy()
    for (j, rr) in [(10, 0), (20, 1), (30, 2), (40, 4)]:
        for unit in (1.0, 1j):
            bp = W.Band(band.ab.copy(), band.n, band.kl, band.ku)
            bm = W.Band(band.ab.copy(), band.n, band.kl, band.ku)
            bp.ab[j, rr] += unit * h
            bm.ab[j, rr] -= unit * h
            d = np.sum(sig(z, bp) - sig(z, bm)) / (2 * h)
            got = gbn[j, rr].real if unit == 1.0 else gbn[j, rr].imag
            assert abs(got - d) < 2e-6, (j, rr, unit, got, d)


def test_newton_contour_circles():
    api = _api()
    import torch
    a = np.array([0.4 + 0.1j, 5.0, -5.0])
    band = W.diagonal(a)
    mat = api.BandedMatrix.from_band(band)
    eps = 1e-3
    # Newton on ln(r/eps) maps r -> r (1 - ln(r/eps)): three steps from within 30 % of eps
    # reach 1e-6; from 2 eps it takes six.
    z0 = a[0] + np.array([1.3e-3, 0.8e-3j, -1.1e-3 - 0.4e-3j, 0.75e-3 * np.exp(0.3j)])
    z, s = api.newton_contour(mat, torch.tensor(z0, dtype=torch.complex128, device="cuda"), eps, steps=3)
    np.testing.assert_allclose(np.abs(z.cpu().numpy() - a[0]), eps, rtol=1e-6)
    np.testing.assert_allclose(s.cpu().numpy(), eps, rtol=1e-6)
    z, s = api.newton_contour(mat, torch.tensor([a[0] + 2e-3], dtype=torch.complex128, device="cuda"), eps, steps=6)
    np.testing.assert_allclose(s.cpu().numpy(), eps, rtol=1e-6)


def test_sigmamin_autograd_function():
    api = _api()
    import torch
    band = W.grcar(40)
    ab = torch.tensor(band.ab, dtype=torch.complex128, device="cuda", requires_grad=True)
    z = torch.tensor([0.5 + 1.5j, 2.0 - 1.0j], dtype=torch.complex128, device="cuda", requires_grad=True)
    mat = api.BandedMatrix.from_band(band)
    s = api.SigmaMin.apply(ab, z, mat)
    loss = (s * torch.tensor([1.0, -2.0], device="cuda", dtype=torch.float64)).sum()
    loss.backward()
    r = api.sigma_min(mat, z.detach(), want_vectors=True)
    gz, gb = api.backward(mat, torch.tensor([1.0, -2.0], dtype=torch.float64, device="cuda"), r["u"], r["v"])
    np.testing.assert_allclose(z.grad.cpu().numpy(), gz.cpu().numpy(), atol=1e-8)
    np.testing.assert_allclose(ab.grad.cpu().numpy(), gb.cpu().numpy(), atol=1e-8)


def test_sigmamin_follows_an_edited_band():
    """SigmaMin with a band tensor whose values differ from the handle's (edited in place after
    the handle was built): sigma and both gradients are those of the edited matrix, equal to a
    fresh handle's; with the band unchanged the handle is used as it is."""
    api = _api()
    import torch
    band = W.grcar(40)
    mat = api.BandedMatrix.from_band(band)
    ab = torch.tensor(band.ab, dtype=torch.complex128, device="cuda")
    ab[5, band.ku] += 0.75                  # A[5][5] += 0.75, after mat was built
    ab.requires_grad_(True)
    z = torch.tensor([0.5 + 1.5j, 2.0 - 1.0j, 1.2 + 0.1j], dtype=torch.complex128, device="cuda", requires_grad=True)
    w = torch.tensor([1.0, -2.0, 0.5], device="cuda", dtype=torch.float64)
    s = api.SigmaMin.apply(ab, z, mat)
    (s * w).sum().backward()
    fresh = api.BandedMatrix(ab.detach(), band.n, band.kl, band.ku, real=mat.real)   # the edit keeps A real
    r = api.sigma_min(fresh, z.detach(), want_vectors=True)
    gz, gb = api.backward(fresh, w, r["u"], r["v"])
    old = api.sigma_min(mat, z.detach())["sigma"]
    assert not torch.allclose(old, r["sigma"])            # the edit changes sigma
    np.testing.assert_array_equal(s.detach().cpu().numpy(), r["sigma"].cpu().numpy())
    np.testing.assert_allclose(z.grad.cpu().numpy(), gz.cpu().numpy(), atol=1e-8)
    np.testing.assert_allclose(ab.grad.cpu().numpy(), gb.cpu().numpy(), atol=1e-8)
    with pytest.raises(ValueError):
        api.SigmaMin.apply(ab.detach()[:-1], z.detach(), mat)


def test_contour_seeds_vs_oracle():
    """ps_contour_seeds on the grcar100 grid (the GPU's own sigma values feed both sides, so
    the sign decisions are the same): same edges in the same order, same points."""
    api = _api()
    import torch
    w = W.workload("grcar100")
    mat = api.BandedMatrix.from_band(w["band"])
    grid = w["grid"]
    r = api.eval_grid(mat, grid)
    sig = r["sigma"].cpu().numpy()
    for eps in (1e-1, 1e-3, 1e-6):
        seeds, count = api.contour_seeds(grid, r["sigma"], eps)
        ref = oracle.contour_seeds(grid, sig, eps)
        assert count == len(ref) > 0, (eps, count, len(ref))
        np.testing.assert_allclose(seeds.cpu().numpy(), ref, rtol=0, atol=1e-13)
    # capacity below the count: the first max_seeds in edge order, the full count reported
    seeds, count = api.contour_seeds(grid, r["sigma"], 1e-3, max_seeds=7)
    assert count == len(oracle.contour_seeds(grid, sig, 1e-3)) and seeds.numel() == 7
    np.testing.assert_allclose(seeds.cpu().numpy(), oracle.contour_seeds(grid, sig, 1e-3)[:7], rtol=0, atol=1e-13)
    # ragged sizes: a single row and a single column (only one kind of edge)
    for g in (W.Grid(-1.0, 3.0, 0.5, 0.5, 37, 1), W.Grid(0.2, 0.2, -3.0, 3.0, 1, 29)):
        rr = api.eval_grid(mat, g)
        s = rr["sigma"].cpu().numpy()
        seeds, count = api.contour_seeds(g, rr["sigma"], 1e-2)
        ref = oracle.contour_seeds(g, s, 1e-2)
        assert count == len(ref)
        np.testing.assert_allclose(seeds.cpu().numpy(), ref, rtol=0, atol=1e-13)
