"""CPU tests of the classifier's training copy and of the matrix features (Sec. 3.1, 3.2): the
torch network equals the oracle's network within the oracle's float32 error bound, the folded
standardisation exports the same function, and the features meet closed forms."""
import numpy as np
import pytest

import oracle.mask as om
import workloads as W
from workloads import nets

torch = pytest.importorskip("torch")


def test_torch_network_matches_oracle():
    from paper_2605_04550_amd.train_mask import MaskMLP, NPARAM
    assert NPARAM == om.NPARAM
    params = nets.mlp_params(71, 3.0)
    rng = np.random.default_rng(5)
    gf = rng.standard_normal(30)
    eig = nets.spectrum(72, 40)
    z = rng.uniform(-4, 4, 200) + 1j * rng.uniform(-4, 4, 200)
    ref, bnd = om.mlp_prob(params, gf, eig, z, bound=True)
    net = MaskMLP()
    net.load_flat(params)
    g = om.point_features(z, eig)
    feat = torch.tensor(np.concatenate([np.broadcast_to(gf, (200, 30)), g], axis=1), dtype=torch.float32)
    phi = MaskMLP.fourier(torch.tensor(z.real, dtype=torch.float32), torch.tensor(z.imag, dtype=torch.float32))
    with torch.no_grad():
        p = torch.sigmoid(net(phi, feat)).double().numpy()
    # the torch inputs are float32 roundings of the features, which the bound counts
    assert np.all(np.abs(p - ref) <= bnd), np.max(np.abs(p - ref) / bnd)
    assert np.array_equal(net.export(), params)


def test_folded_standardisation_exports_the_same_function():
    from paper_2605_04550_amd.train_mask import MaskMLP
    torch.manual_seed(3)
    net = MaskMLP().double()
    rng = np.random.default_rng(9)
    raw = rng.standard_normal((50, 33)) * rng.uniform(0.1, 5.0, 33) + rng.uniform(-3, 3, 33)
    mu, sd = raw.mean(axis=0), raw.std(axis=0)
    phi = torch.tensor(rng.standard_normal((50, 26)))
    with torch.no_grad():
        a = net(phi, torch.tensor((raw - mu) / sd)).numpy()
        flat = net.export(mu, sd).astype(np.float64)
        net2 = MaskMLP().double()
        p = np.asarray(flat)
        at = 0
        for name, o, i in [("c1", 64, 26), ("c2", 64, 64), ("m1", 128, 33), ("m2", 64, 128), ("r4", 128, 128),
                           ("r5", 128, 128), ("p7", 64, 128), ("out", 1, 64)]:
            net2.lin[name].weight.copy_(torch.tensor(p[at:at + o * i].reshape(o, i)))
            at += o * i
            net2.lin[name].bias.copy_(torch.tensor(p[at:at + o]))
            at += o
        b = net2(phi, torch.tensor(raw)).numpy()
    # the export rounds to float32: agreement to float32 accuracy of the logits
    assert np.max(np.abs(a - b)) <= 1e-4 * (1 + np.max(np.abs(a)))


def test_global_features_closed_forms():
    from paper_2605_04550_amd.features import global_features
    n = 8
    d = 1.0 + 1.13 * np.arange(n)            # no eigenvalue at the centroid + 0.5, 1, 2
    dmax = d[-1]
    f, lam = global_features(np.diag(d), seed=1)
    assert np.allclose(np.sort(lam.real), d) and np.allclose(lam.imag, 0)
    assert np.isclose(f[0], d.mean()) and np.isclose(f[1], d.std()) and f[2] == 1 and np.isclose(f[3], dmax)
    assert np.allclose(f[4:8], 0) and np.isclose(f[8], dmax) and np.isclose(f[9], 1)
    assert f[10] == 0 and f[11] == 0                                  # normal: A = A^T = A^H
    assert np.isclose(f[12], np.log10(dmax + 1e-12))
    fro = np.linalg.norm(d)
    assert np.isclose(f[13], dmax / fro) and np.isclose(f[14], dmax / fro) and np.isclose(f[15], dmax / fro)
    assert np.isclose(f[16], d.mean()) and np.isclose(f[17], d.std()) and f[18] == 0 and f[19] == 0
    assert np.isclose(f[20], 1.0 / n)
    assert np.isclose(f[21], np.sum((d / fro) ** 2) / n ** 2)
    assert abs(f[23]) < 1e-10                                         # kappa(V) = 1
    assert np.isclose(f[24], np.log10(1e-12))
    assert np.isclose(f[25], (dmax - 1.0) / dmax) and np.isclose(f[26], (dmax - 1.0) / dmax)
    # resolvent at the centroid + delta: for a diagonal matrix |x| / |b| is a weighted mean of
    # 1 / |c + delta - d_i|, between its smallest and largest value
    c = d.mean()
    for k, delta in enumerate((0.5, 1.0, 2.0)):
        r = 1.0 / np.abs(c + delta - d)
        assert np.log10(r.min()) - 1e-12 <= f[27 + k] <= np.log10(r.max()) + 1e-12
    # a non-normal 2 x 2: ||A - A^T||_F / ||A||_F
    A = np.array([[1.0, 2.0], [0.0, 3.0]])
    f2, _ = global_features(A)
    assert np.isclose(f2[10], np.sqrt(8.0) / np.sqrt(14.0)) and np.isclose(f2[11], f2[10])
    assert np.isclose(f2[20], 0.75)


def test_balanced_sampling_rule():
    from paper_2605_04550_amd.train_mask import balanced_samples
    lab = np.zeros((4, 50, 50), dtype=np.uint8)
    lab[0, :5, :6] = 1          # 30 positives -> 300 negatives
    lab[1, 0, 0] = 1            # 1 positive -> 200 negatives
    lab[3, :48, :] = 1          # 2400 positives -> all 100 negatives there are
    s = balanced_samples(dict(labels=lab), np.random.default_rng(0))
    for m, want_pos, want_neg in [(0, 30, 300), (1, 1, 200), (2, 0, 200), (3, 2400, 100)]:
        rows = s[s[:, 0] == m, 1]
        flat = lab[m].ravel()
        assert np.sum(flat[rows] == 1) == want_pos and np.sum(flat[rows] == 0) == want_neg
        assert len(np.unique(rows)) == len(rows)
