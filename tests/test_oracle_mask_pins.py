"""Pins for the mask-producer oracle (``oracle/mask.py``, Sec. 3.2 and Sec. 3.5).

Each pin is independent of the oracle's own code: closed forms of the Fourier features and of
the eigenvalue-distance features, brute force, the network rebuilt from torch.nn layers (a
library implementation of the dense layers, SiLU and the sigmoid), a float32 evaluation
checked against the oracle's error bound, numpy's quantile, and the cell selection and
dilation rebuilt from np.kron and scipy.ndimage.  ``test_mask_oracle_mutants`` plants
mistakes in copies of the oracle and checks that these pins catch each one.
"""
import importlib.util
import math
import os
import tempfile

import numpy as np
import pytest

import workloads as W
from oracle import mask as M0
from workloads import nets

ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "mask.py")


# ----------------------------------------------------------------------------- features

def pin_fourier_closed_form(M):
    # x = pi/4: sin(2x) = 1, cos(2x) = 0, sin(4x) = 0, cos(4x) = -1, then sin = 0, cos = 1.
    # y = pi/8: sin(2y) = cos(2y) = 1/sqrt2, sin(4y) = 1, cos(4y) = 0, sin(8y) = 0,
    # cos(8y) = -1, then sin = 0, cos = 1.
    x, y = math.pi / 4, math.pi / 8
    r = 1 / math.sqrt(2)
    expect = [x, y,
              1, r, 0, r,          # sin(2c), cos(2c)
              0, 1, -1, 0,         # sin(4c), cos(4c)
              0, 0, 1, -1,         # sin(8c), cos(8c)
              0, 0, 1, 1,          # 16
              0, 0, 1, 1,          # 32
              0, 0, 1, 1]          # 64
    got = M.fourier_features(np.array([x]), np.array([y]))[0]
    assert got.shape == (26,)
    np.testing.assert_allclose(got, expect, atol=1e-13)


def pin_point_features(M):
    eig = np.array([1, -1, 1j, -1j])
    g = M.point_features(np.array([0.0, 2.0]), eig)
    np.testing.assert_allclose(g[0], [1.0, 0.0, 1.0], atol=1e-15)
    np.testing.assert_allclose(g[1], [1.0, 2.0, (1 + 3 + 2 * math.sqrt(5)) / 4], atol=1e-15)
    # brute force on a random spectrum
    rng = np.random.default_rng(11)
    eig = rng.standard_normal(37) + 1j * rng.standard_normal(37)
    z = rng.standard_normal(9) + 1j * rng.standard_normal(9)
    g = M.point_features(z, eig)
    cx = sum(e.real for e in eig) / len(eig)
    cy = sum(e.imag for e in eig) / len(eig)
    for p in range(len(z)):
        ds = [math.hypot(z[p].real - e.real, z[p].imag - e.imag) for e in eig]
        assert abs(g[p, 0] - min(ds)) < 1e-14
        assert abs(g[p, 1] - math.hypot(z[p].real - cx, z[p].imag - cy)) < 1e-14
        assert abs(g[p, 2] - sum(ds) / len(ds)) < 1e-13


def test_fourier_closed_form():
    pin_fourier_closed_form(M0)


def test_point_features():
    pin_point_features(M0)


# ----------------------------------------------------------------------------- the network

def _torch_prob(params, gfeat, eig, z):
    """The dual-path network of Sec. 3.2 assembled from torch.nn.Linear layers (float64)."""
    import torch
    import torch.nn as nn
    p = torch.tensor(np.asarray(params, dtype=np.float64))
    layers, at = [], 0
    for o, i in nets.LAYER_SHAPES:
        lin = nn.Linear(i, o).double()
        with torch.no_grad():
            lin.weight.copy_(p[at:at + o * i].reshape(o, i))
            at += o * i
            lin.bias.copy_(p[at:at + o])
            at += o
        layers.append(lin)
    c1, c2, m1, m2, r4, r5, p7, out = layers
    silu = nn.functional.silu
    zt = torch.tensor(np.asarray(z, dtype=np.complex128))
    c = torch.stack([zt.real, zt.imag], dim=1)
    enc = [c]
    for k in range(1, 7):
        enc += [torch.sin(2.0 ** k * c), torch.cos(2.0 ** k * c)]
    phi = torch.cat(enc, dim=1)
    lam = torch.tensor(np.asarray(eig, dtype=np.complex128))
    d = (zt[:, None] - lam[None, :]).abs()
    g = torch.stack([d.min(dim=1).values, (zt - lam.mean()).abs(), d.mean(dim=1)], dim=1)
    f = torch.cat([torch.tensor(gfeat, dtype=torch.float64).expand(len(zt), 30), g], dim=1)
    hc = silu(c2(silu(c1(phi))))
    hm = silu(m2(silu(m1(f))))
    h4 = silu(r4(torch.cat([hc, hm], dim=1)))
    h6 = h4 + silu(r5(h4))
    h7 = silu(p7(h6))
    with torch.no_grad():
        return torch.sigmoid(out(h7))[:, 0].numpy()


def _inputs(k, m=40, scale=3.0, n=23):
    rng = np.random.default_rng(300 + k)
    z = rng.uniform(-4, 4, m) + 1j * rng.uniform(-4, 4, m)
    return nets.mlp_params(40 + k, scale), nets.global_features(50 + k), nets.spectrum(60 + k, n), z


def pin_network_vs_torch(M):
    for k in range(3):
        params, gf, eig, z = _inputs(k)
        p = M.mlp_prob(params, gf, eig, z)
        ref = _torch_prob(params, gf, eig, z)
        np.testing.assert_allclose(p, ref, rtol=0, atol=1e-12)
        assert p.std() > 0.05          # the draws spread p: the comparison is not vacuous


def pin_network_constant(M):
    # every weight zero: each hidden layer is SiLU of its bias and p = sigmoid(b_out)
    params = np.zeros(nets.NPARAM, dtype=np.float32)
    params[-1] = 0.75
    p = M.mlp_prob(params, np.zeros(30), np.array([0j]), np.array([0.3 + 0.1j, -2 + 3j]))
    np.testing.assert_allclose(p, 1 / (1 + math.exp(-0.75)), rtol=1e-15)


def _f32_prob(M, params, gfeat, eig, z):
    """float32 evaluation (numpy float32 matmul and elementwise ops)."""
    f32 = np.float32
    L = {k: (W.astype(f32), b.astype(f32)) for k, (W, b) in M.unpack(params).items()}
    m = len(z)
    phi = M.fourier_features(z.real, z.imag).astype(f32)
    feat = np.concatenate([np.broadcast_to(gfeat, (m, 30)), M.point_features(z, eig)], axis=1).astype(f32)

    def dense(k, h):
        Wk, bk = L[k]
        return (h @ Wk.T + bk).astype(f32)

    def silu(x):
        with np.errstate(over="ignore"):
            return (x / (f32(1) + np.exp(-x))).astype(f32)

    hc = silu(dense("c2", silu(dense("c1", phi))))
    hm = silu(dense("m2", silu(dense("m1", feat))))
    h4 = silu(dense("r4", np.concatenate([hc, hm], axis=1)))
    h6 = (h4 + silu(dense("r5", h4))).astype(f32)
    zl = dense("out", silu(dense("p7", h6)))[:, 0]
    with np.errstate(over="ignore"):
        return (f32(1) / (f32(1) + np.exp(-zl))).astype(np.float64)


def pin_error_bound(M):
    for k in range(3):
        params, gf, eig, z = _inputs(k, m=200)
        p, e = M.mlp_prob(params, gf, eig, z, bound=True)
        p32 = _f32_prob(M, params, gf, eig, z)
        assert np.all(np.abs(p32 - p) <= e), np.max(np.abs(p32 - p) / e)
        # not vacuous: weights of this scale make p sensitive, and the bound sums the worst
        # case of every rounding site, yet it stays far below the spread of p
        assert np.median(e) < 5e-3 and np.max(e) < 2e-2


def pin_bound_vs_autograd(M):
    import torch
    params, gf, eig, z = _inputs(1, m=30)
    _, e = M.mlp_prob(params, gf, eig, z, bound=True)
    # sensitivities from autograd on the full (non-detached) graph
    u = 2.0 ** -24
    p = torch.tensor(np.asarray(params, dtype=np.float64))
    Ws, at = [], 0
    for o, i in nets.LAYER_SHAPES:
        Ws.append((p[at:at + o * i].reshape(o, i), p[at + o * i:at + o * i + o]))
        at += o * i + o
    zt = torch.tensor(np.asarray(z, dtype=np.complex128))
    c = torch.stack([zt.real, zt.imag], dim=1)
    phi = torch.cat([c] + [fn(2.0 ** k * c) for k in range(1, 7) for fn in (torch.sin, torch.cos)], dim=1)
    lam = torch.tensor(np.asarray(eig, dtype=np.complex128))
    d = (zt[:, None] - lam[None, :]).abs()
    g = torch.stack([d.min(dim=1).values, (zt - lam.mean()).abs(), d.mean(dim=1)], dim=1)
    f = torch.cat([torch.tensor(gf, dtype=torch.float64).expand(len(zt), 30), g], dim=1)
    sites = []

    def keep(x, loc):
        x.retain_grad()
        sites.append((x, loc))
        return x

    def lin(k, h):
        W, b = Ws[k]
        K = W.shape[1] + 1
        return keep(h @ W.T + b, K * u / (1 - K * u) * (h.detach().abs() @ W.abs().T + b.abs()))

    def act(y, fn=torch.nn.functional.silu):
        a = fn(y)
        return keep(a, (4 * (1 + y.detach().abs()) + 4) * u * a.detach().abs())

    x1 = keep(phi.clone().requires_grad_(True), 1.01 * u * phi.abs())
    x2 = keep(f.clone().requires_grad_(True), 1.01 * u * f.abs())
    hc = act(lin(1, act(lin(0, x1))))
    hm = act(lin(3, act(lin(2, x2))))
    h4 = act(lin(4, torch.cat([hc, hm], dim=1)))
    h6 = keep(h4 + act(lin(5, h4)), None)
    sites[-1] = (h6, u * h6.detach().abs())
    pr = act(lin(7, act(lin(6, h6))), torch.sigmoid)
    pr.sum().backward()
    ref = 2 * sum((x.grad.abs() * loc).sum(dim=1) for x, loc in sites).numpy()
    np.testing.assert_allclose(e, ref, rtol=1e-10)


def test_bound_vs_autograd():
    pin_bound_vs_autograd(M0)


def test_network_vs_torch():
    pin_network_vs_torch(M0)


def test_network_constant():
    pin_network_constant(M0)


def test_error_bound_covers_float32():
    pin_error_bound(M0)


def test_parameter_count_is_the_paper_shapes():
    # Sec. 3.2 layer shapes: 1728 + 4160 + 4352 + 8256 + 2 * 16512 + 8256 + 65
    assert M0.NPARAM == nets.NPARAM == 59841
    assert tuple((o, i) for _, o, i in M0.LAYERS) == nets.LAYER_SHAPES


# ----------------------------------------------------------------------------- hierarchy

def pin_quantile(M):
    rng = np.random.default_rng(5)
    for m in list(range(1, 40)) + [624, 625, 626, 2501]:
        v = rng.uniform(size=m).astype(np.float32).astype(np.float64)
        got = M.quantile_linear(v, 0.8)
        ref = np.quantile(v, 0.8, method="linear")
        assert abs(got - ref) <= 4 * np.spacing(ref), (m, got, ref)
        if (m - 1) % 5 == 0:                      # 0.8 (m - 1) an integer: an order statistic
            assert got == np.sort(v)[int(round(0.8 * (m - 1)))]
    v = np.array([0.1, 0.3, 0.3, 0.3, 0.9])
    assert M.quantile_linear(v, 0.8) == pytest.approx(0.3 + 0.2 * 0.6, abs=1e-15)   # h = 3.2


def _hashed_prob(grid, seed):
    table = np.random.default_rng(seed).uniform(size=grid.npts)
    return lambda flat: table[np.asarray(flat, dtype=np.int64)], table


def pin_hierarchy(M):
    from scipy import ndimage
    cases = [(W.Grid(-4, 4, -4, 4, 100, 100), 4, 5, 0.5), (W.Grid(-1, 2, 0, 3, 37, 23), 4, 5, 0.3),
             (W.Grid(0, 1, 0, 1, 50, 61), 8, 3, 0.6), (W.Grid(0, 1, 0, 1, 17, 9), 2, 7, 0.4),
             (W.Grid(0, 1, 0, 1, 1, 1), 4, 5, 0.1), (W.Grid(0, 1, 0, 0, 13, 1), 4, 1, 0.5),
             (W.Grid(0, 0, 0, 1, 1, 30), 3, 5, 0.2)]
    for k, (g, s, dil, tau) in enumerate(cases):
        prob_at, table = _hashed_prob(g, 70 + k)
        r = M.hierarchical_mask(g, prob_at, tau, stride=s, q=0.8, dilate=dil)
        full = table.reshape(g.ny, g.nx)
        coarse = full[::s, ::s]
        np.testing.assert_array_equal(r["coarse"], coarse)
        tc = np.quantile(coarse, 0.8, method="linear")
        assert abs(r["tau_coarse"] - tc) <= 4 * np.spacing(tc)
        sel = coarse >= r["tau_coarse"]
        np.testing.assert_array_equal(r["selected"], sel)
        fine_sel = np.kron(sel, np.ones((s, s), dtype=bool))[:g.ny, :g.nx]
        np.testing.assert_array_equal(r["prob"], np.where(fine_sel, full, 0.0))
        exp_mask = ndimage.binary_dilation(np.where(fine_sel, full, 0.0) >= tau, structure=np.ones((dil, dil)))
        np.testing.assert_array_equal(r["mask"], exp_mask.astype(np.uint8))
        assert r["evals"] == coarse.size + int(fine_sel.sum())


def test_quantile_vs_numpy():
    pin_quantile(M0)


def test_hierarchy_vs_kron_and_scipy():
    pin_hierarchy(M0)


def test_paper_grid_evaluation_count():
    # Sec. 3.5: 100 x 100 grid, stride 4 -> 625 coarse points; the 80th percentile keeps
    # 125 cells (distinct values) -> 625 + 16 * 125 = 2625 evaluations
    g = W.Grid(-4, 4, -4, 4, 100, 100)
    prob_at, _ = _hashed_prob(g, 3)
    r = M0.hierarchical_mask(g, prob_at, 0.05)
    assert r["selected"].sum() == 125 and r["evals"] == 2625


def test_mask_predict_is_the_network_through_the_hierarchy():
    params, gf, eig, _ = _inputs(0)
    g = W.Grid(-4, 4, -4, 4, 30, 26)
    r = M0.mask_predict(params, gf, eig, g, 0.5)

    def prob_at(flat):
        return M0.mlp_prob(params, gf, eig, M0.mask_points_z(g, flat))
    r2 = M0.hierarchical_mask(g, prob_at, 0.5)
    np.testing.assert_array_equal(r["mask"], r2["mask"])
    np.testing.assert_array_equal(r["prob"], r2["prob"])
    z = M0.mask_points_z(g, np.arange(g.npts))
    np.testing.assert_allclose(z.reshape(g.ny, g.nx)[3, 7], complex(-4 + 8 * 7 / 29, -4 + 8 * 3 / 25), atol=1e-15)


def pin_calibration(M):
    from scipy import ndimage
    rng = np.random.default_rng(17)
    nval, ny, nx = 9, 23, 31
    prob = rng.uniform(size=(nval, ny, nx)) ** 13                  # mostly small, a few near 1
    labels = (rng.uniform(size=(nval, ny, nx)) < 0.03).astype(np.uint8)
    labels[4] = 0                                                   # a matrix with no sensitive point
    taus = np.round(np.arange(0.05, 0.95, 0.01), 2)
    r = M.calibrate_tau(prob, labels, taus)
    for m in range(nval):
        lab = ndimage.binary_dilation(labels[m] != 0, structure=np.ones((3, 3)))
        for k in (0, 10, 45, 89):
            if lab.sum() == 0:
                assert r["recall"][m, k] == 1.0
                continue
            pred = ndimage.binary_dilation(prob[m] >= taus[k], structure=np.ones((5, 5)))
            assert r["recall"][m, k] == (pred & lab).sum() / lab.sum()
    np.testing.assert_allclose(r["median"], np.median(r["recall"], axis=0), rtol=0, atol=1e-15)
    np.testing.assert_allclose(r["p10"], np.percentile(r["recall"], 10, axis=0), rtol=0, atol=1e-15)
    ok = (np.median(r["recall"], axis=0) >= 0.9) & (np.percentile(r["recall"], 10, axis=0) >= 0.75)
    assert r["index"] == (int(np.argmax(ok)) if ok.any() else -1) == 0
    assert r["index_max"] == len(taus) - 1 - int(np.argmax(ok[::-1]))
    assert 0 < r["index_max"] < len(taus) - 1                      # the draws put it inside the range
    assert ok[:r["index_max"] + 1].all() and not ok[r["index_max"] + 1:].any()
    # recall falls as tau rises (fewer predicted points)
    assert np.all(np.diff(r["recall"], axis=1) <= 0)
    # closed form: one label point, one predicted point at Chebyshev distance d: the dilated
    # sets (radii 2 and 1) meet the 3 x 3 label square in (4 - d) columns when d <= 3
    for d in range(0, 5):
        p = np.zeros((1, 15, 15))
        lb = np.zeros((1, 15, 15), dtype=np.uint8)
        lb[0, 7, 7] = 1
        p[0, 7, 7 + d] = 0.5
        rr = M.calibrate_tau(p, lb, [0.5, 0.6])
        assert rr["recall"][0, 0] == max(0, min(3, 4 - d)) * 3 / 9, d
        assert rr["recall"][0, 1] == 0.0


def test_calibration():
    pin_calibration(M0)


# ----------------------------------------------------------------------------- mutants

PINS = [pin_fourier_closed_form, pin_point_features, pin_network_vs_torch, pin_network_constant,
        pin_error_bound, pin_bound_vs_autograd, pin_quantile, pin_hierarchy, pin_calibration]

MUTANTS = [
    ("sin/cos order", "cols += [np.sin(f * x), np.sin(f * y), np.cos(f * x), np.cos(f * y)]",
     "cols += [np.cos(f * x), np.cos(f * y), np.sin(f * x), np.sin(f * y)]"),
    ("frequency 2^(k-1)", "f = float(2 ** k)", "f = float(2 ** (k - 1))"),
    ("lambda* = nearest", "np.abs(z - cent)", "d.min(axis=1)"),
    ("dropped bias", "        return h @ W.T + b\n", "        return h @ W.T\n"),
    ("transposed W", "        return h @ W.T + b\n", "        return h @ W.reshape(W.shape[::-1]) + b\n"),
    ("concat order", "h3 = np.concatenate([hc2, hm2], axis=1)", "h3 = np.concatenate([hm2, hc2], axis=1)"),
    ("residual from h3", "h6 = h4 + h5 ", "h6 = h5 + h3[:, :h5.shape[1]] "),
    ("missing SiLU", "h7 = _silu(y7)", "h7 = y7"),
    ("quantile without interpolation", "return v0 + g * (v1 - v0)", "return v0"),
    ("strict selection", "selected = coarse >= tau_c", "selected = coarse > tau_c"),
    ("dilation radius", "r = (dilate - 1) // 2", "r = (dilate + 1) // 2"),
    ("bound without the dense layers", "np.abs(g_y5) * local(\"r5\", h4)", "0.0 * local(\"r5\", h4)"),
    ("recall without the label dilation", "lab = dilate(labels[m] != 0, label_dilate)", "lab = labels[m] != 0"),
    ("recall of an empty label set", "                recall[m, k] = 1.0\n", "                recall[m, k] = 0.0\n"),
    ("tau* as the largest", "index=int(ok[0]) if ok.size", "index=int(ok[-1]) if ok.size"),
    ("median for P10", "p10 = np.array([quantile_linear(recall[:, k], 0.1)", "p10 = np.array([quantile_linear(recall[:, k], 0.5)"),
    ("bound without the inputs", "e += np.sum(np.abs(g_x) * 1.01 * U32 * np.abs(x), axis=1)", "pass"),
]


def _load_mutant(src, tag):
    d = tempfile.mkdtemp()
    path = os.path.join(d, "mask_mutant.py")
    with open(path, "w") as f:
        f.write(src)
    spec = importlib.util.spec_from_file_location("mask_mutant_" + tag, path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mask_oracle_mutants(name, old, new):
    src = open(ORACLE_SRC).read()
    assert src.count(old) == 1, name
    mod = _load_mutant(src.replace(old, new), str(abs(hash(name))))
    caught = []
    for pin in PINS:
        try:
            pin(mod)
        except Exception:                # AssertionError or a shape error
            caught.append(pin.__name__)
    assert caught, "mutant '%s' survives every pin" % name
