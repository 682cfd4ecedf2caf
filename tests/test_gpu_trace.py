"""GPU parity of eps-contour tracing (ps_trace_contour): a tangent step of length h along the
eps-level curve of sigma_min (the boundary the paper draws as the level curve log10 eps,
Sec. 2.1), then Newton corrections.  Checked against the closed form of a normal matrix
(circles), against the oracle's tracer step by step, and by re-evaluating sigma_min at the
traced points."""
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


def test_trace_circles_closed_form():
    api = _api()
    import torch
    import paper_2605_04550_amd as P
    a = np.array([0.4 + 0.1j, -0.3 - 0.2j, 5.0])
    mat = api.BandedMatrix.from_band(W.diagonal(a))
    eps, h = 1e-2, 1e-3
    seeds = torch.tensor([a[0] + 1.2e-2, a[1] - 0.9e-2j], dtype=torch.complex128, device="cuda")
    r = api.trace_contour(mat, seeds, eps, h, 200)
    cnt, fl = r["count"].cpu().numpy(), r["flags"].cpu().numpy()
    pts = r["points"].cpu().numpy()
    assert list(fl) == [P.PS_TRACE_CLOSED, P.PS_TRACE_CLOSED]
    th = np.arctan(h / eps)
    for t in range(2):
        p = pts[t, :cnt[t]]
        assert np.all(np.abs(np.abs(p - a[t]) - eps) < 1e-10)
        np.testing.assert_allclose(np.abs(np.diff(p)), 2 * eps * np.sin(th / 2), rtol=1e-6)
        assert abs(cnt[t] - 2 * np.pi / th) <= 2
        assert np.all(np.diff(np.unwrap(np.angle(p - a[t]))) > 0)       # counterclockwise
    box = (a[0].real - 1.0, a[0].real + 1.0, a[0].imag - 1.0, a[0].imag + 0.005)
    r = api.trace_contour(mat, seeds[:1], eps, h, 200, box=box)
    assert int(r["flags"][0]) == P.PS_TRACE_LEFT_BOX
    r = api.trace_contour(mat, seeds[:1], eps, h, 10)
    assert int(r["flags"][0]) == P.PS_TRACE_MAX_POINTS and int(r["count"][0]) == 10


def test_trace_matches_oracle_tracer_grcar():
    """Same seeds, same steps: the GPU and oracle tracers stay together point by point (each
    point is pulled back onto the curve; only the position along it can drift, by the
    rounding of the tangent)."""
    api = _api()
    import torch
    band = W.grcar(60)
    mat = api.BandedMatrix.from_band(band)
    eps, h = 1e-2, 0.02
    seeds = np.array([0.3 + 1.9j, 2.2 - 0.7j, 1.0 + 2.3j])
    pts_o, cnt_o, fl_o = oracle.trace_contour(band, seeds, eps, h, max_points=20)
    r = api.trace_contour(mat, torch.tensor(seeds, dtype=torch.complex128, device="cuda"), eps, h, 20)
    cnt, fl = r["count"].cpu().numpy(), r["flags"].cpu().numpy()
    pts = r["points"].cpu().numpy()
    assert np.array_equal(cnt, cnt_o) and np.array_equal(fl, fl_o), (cnt, cnt_o, fl, fl_o)
    for t in range(len(seeds)):
        err = np.abs(pts[t, :cnt[t]] - pts_o[t, :cnt[t]])
        print("seed %d: %d points, max |z_gpu - z_oracle| %.2e" % (t, cnt[t], err.max()))
        assert np.all(err <= 1e-7), (t, err.max())
        s = oracle.sigma_min(band, pts[t, :cnt[t]])["sigma"]
        assert np.all(np.abs(s - eps) <= tol(band.fro, eps) + 1e-6 * eps)


def test_trace_from_grid_seeds_grcar100():
    """Seeds from ps_contour_seeds on the grcar100 grid, traced inside the grid box: every
    stored point lies on the curve (sigma_min re-evaluated on the GPU and by the oracle)."""
    api = _api()
    import torch
    w = W.workload("grcar100")
    mat = api.BandedMatrix.from_band(w["band"])
    g = w["grid"]
    eps = 1e-3
    r = api.eval_grid(mat, g)
    seeds, count = api.contour_seeds(g, r["sigma"], eps)
    pick = seeds[:: max(1, count // 8)][:8]
    h = 0.5 * (g.b - g.a) / (g.nx - 1)
    tr = api.trace_contour(mat, pick, eps, h, 64, box=(g.a, g.b, g.c, g.d))
    cnt = tr["count"].cpu().numpy()
    fl = tr["flags"].cpu().numpy()
    assert np.all(cnt >= 1) and np.all(fl != 0)
    pts = np.concatenate([tr["points"][t, :cnt[t]].cpu().numpy() for t in range(len(cnt))])
    s_gpu = api.sigma_min(mat, torch.tensor(pts, dtype=torch.complex128, device="cuda"))["sigma"].cpu().numpy()
    # accepted at |ln(sigma / eps)| <= 1e-6 by the tracer's own evaluation; a second evaluation
    # may differ from it by the evaluation tolerance twice (each within tol of the truth)
    worst = float(np.max(np.abs(s_gpu - eps)))
    print("grcar100: max |sigma - eps| of the stored points %.3e (bound %.3e)"
          % (worst, 1e-6 * eps + 2 * tol(w["band"].fro, eps)), flush=True)
    assert np.all(np.abs(s_gpu - eps) <= 1e-6 * eps + 2 * tol(w["band"].fro, eps))
    sel = np.arange(0, len(pts), max(1, len(pts) // 12))
    s_or = oracle.sigma_min(w["band"], pts[sel])["sigma"]
    assert np.all(np.abs(s_or - eps) <= tol(w["band"].fro, eps) + 1e-6 * eps)
    print("grcar100: %d tracers, %d points, flags %s" % (len(cnt), len(pts), fl.tolist()))


def test_trace_at_the_benchmarked_size_certified():
    """The launch the tracing benchmark times: toeplitz n = 2000, 256 seeds from the eps = 1e-2
    contour seeds of the full 256 x 256 grid, h = the grid spacing, 64 points each.  Sampled
    stored points are certified by the oracle's inertia count: no singular value of zI - A
    below eps - d and at least one below eps + d, d = 1e-6 eps + 2 tol (the acceptance bound
    and the evaluation tolerance)."""
    api = _api()
    w = W.workload("toeplitz2000")
    band, g = w["band"], w["grid"]
    mat = api.BandedMatrix.from_band(band)
    eps = 1e-2
    r = api.eval_grid(mat, g)
    seeds, count = api.contour_seeds(g, r["sigma"], eps)
    pick = seeds[:: max(1, count // 256)][:256].contiguous()
    h = (g.b - g.a) / (g.nx - 1)
    tr = api.trace_contour(mat, pick, eps, h, 64, box=(g.a, g.b, g.c, g.d))
    cnt = tr["count"].cpu().numpy()
    assert len(cnt) == 256 and np.all(cnt >= 1)
    pts = np.concatenate([tr["points"][t, :cnt[t]].cpu().numpy() for t in range(len(cnt))])
    sel = pts[np.linspace(0, len(pts) - 1, 12).astype(int)]
    d = 1e-6 * eps + 2 * tol(band.fro, eps)
    below = oracle.count_below(band, sel, eps - d)
    above = oracle.count_below(band, sel, eps + d)
    print("toeplitz2000 trace: %d tracers, %d points; certified %d sampled points within %.2e of eps"
          % (len(cnt), len(pts), len(sel), d), flush=True)
    assert np.all(below == 0) and np.all(above >= 1), (below, above)
