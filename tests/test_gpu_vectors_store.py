"""GPU test of the two ways the Golub-Kahan path forms the Ritz vector of a call with singular
vectors: from the Lanczos vectors kept by the first pass, or by replaying the Lanczos steps (a
shift that needed more steps than were kept).  A call keeps as many vectors per slot as its
workspace holds beyond the slots' own needs, up to the default that ps_workspace_size asks
room for; the same shifts are evaluated with that workspace (64 kept), with room for 2 and with
none (every shift replays), and must give the same sigma and the same singular pair; the
residuals of the pair are checked against the matrix itself (the sigma of this path against the
oracle: the vector tests at n = 400 and the all-band-shapes test)."""
import numpy as np
import pytest

import workloads as W
from gpu_util import need_gpu

pytestmark = pytest.mark.gpu


def test_kept_vectors_equal_the_replay():
    need_gpu()
    import torch
    from paper_2605_04550_amd import api, ps_workspace_size
    n = 2000
    band = W.grcar(n)
    A = W.to_dense(band)
    mat = api.BandedMatrix.from_band(band)
    # points across the Grcar pseudospectra: inside the curve the smallest singular values are
    # tiny and clustered, and many shifts need far more than 64 Lanczos steps
    rng = np.random.default_rng(4242)
    z = np.concatenate([rng.uniform(-0.5, 2.5, 24) + 1j * rng.uniform(-2.8, 2.8, 24),
                        0.8 + 1j * np.linspace(-2.0, 2.0, 16)])
    zt = torch.tensor(z, dtype=torch.complex128, device="cuda")
    kw = dict(want_vectors=True, bisect=False, tol_rel=1e-12, tol_norm=1e-14)
    o = api.make_opts(1e-14, 1e-12, 3000, True, 0, bisect=False)
    full = ps_workspace_size(mat.handle, len(z), o)
    # one kept vector of every slot: 256 slots (one quantum for 40 shifts) x (round_up(n, 8) + 8)
    # rows x 16 bytes; the default keeps 64
    per_k = 256 * ((n + 7) // 8 * 8 + 8) * 16
    runs = {}
    for kept in (64, 2, 0):
        ws = torch.empty(full - (64 - kept) * per_k, dtype=torch.uint8, device="cuda")
        runs[kept] = api.sigma_min(mat, zt, workspace=ws, **kw)
    it = runs[64]["iters"].cpu().numpy()
    print("kept vectors 64 / 2 / 0: %d shifts, Lanczos steps median %d max %d, %d above 2, %d above 64"
          % (len(z), np.median(it), it.max(), np.sum(it > 2), np.sum(it > 64)), flush=True)
    assert np.sum(it <= 2) >= 1 and np.sum(it > 2) >= 1 and np.sum(it > 64) >= 1   # every way occurs
    ref = runs[0]
    s0 = ref["sigma"].cpu().numpy()
    u0, v0 = ref["u"].cpu().numpy(), ref["v"].cpu().numpy()
    for kept in (64, 2):
        r = runs[kept]
        assert np.array_equal(r["iters"].cpu().numpy(), ref["iters"].cpu().numpy())
        assert np.array_equal(r["info"].cpu().numpy(), ref["info"].cpu().numpy())
        assert np.array_equal(r["sigma"].cpu().numpy(), s0)
        # the same terms in the same order; only the contraction of a multiply-add may differ
        du = np.abs(r["u"].cpu().numpy() - u0).max()
        dv = np.abs(r["v"].cpu().numpy() - v0).max()
        print("kept %d vs replay: max |du| %.3e, max |dv| %.3e" % (kept, du, dv), flush=True)
        assert du < 1e-12 and dv < 1e-12
    # each pair is a singular pair of zI - A to the working accuracy (backward error)
    u1, v1 = runs[64]["u"].cpu().numpy(), runs[64]["v"].cpu().numpy()
    nA = np.linalg.norm(A)
    for p in range(len(z)):
        assert abs(np.linalg.norm(v1[p]) - 1) < 1e-10 and abs(np.linalg.norm(u1[p]) - 1) < 1e-10
        res = np.linalg.norm(z[p] * v1[p] - A @ v1[p] - s0[p] * u1[p])
        assert res <= 1e-8 * nA + 1e-6 * s0[p], (p, res)
