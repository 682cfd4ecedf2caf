"""GPU test of the two ways the Golub-Kahan path forms the Ritz vector of a call with singular
vectors: from the Lanczos vectors kept by the first pass (calls on at most 4096 slots, up to 64
steps) or by replaying the Lanczos steps (larger calls, or a shift that needed more steps than
were kept).  The same shifts are evaluated both ways (an explicit slot count above 4096 forces
the replay) and must give the same sigma and the same singular pair; the residuals of the pair
are checked against the matrix itself (the σ of this path against the oracle: the vector
tests at n = 400 and the all-band-shapes test)."""
import numpy as np
import pytest

import workloads as W
from gpu_util import need_gpu

pytestmark = pytest.mark.gpu


def test_kept_vectors_equal_the_replay():
    need_gpu()
    import torch
    from paper_2605_04550_amd import api
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
    kept = api.sigma_min(mat, zt, **kw)
    replay = api.sigma_min(mat, zt, slots=8192, **kw)
    it = kept["iters"].cpu().numpy()
    print("kept vs replay: %d shifts, Lanczos steps median %d max %d, %d above 64"
          % (len(z), np.median(it), it.max(), np.sum(it > 64)), flush=True)
    assert np.sum(it <= 64) >= 1 and np.sum(it > 64) >= 1       # both ways occur
    assert np.array_equal(it, replay["iters"].cpu().numpy())
    assert np.array_equal(kept["info"].cpu().numpy(), replay["info"].cpu().numpy())
    s1, s2 = kept["sigma"].cpu().numpy(), replay["sigma"].cpu().numpy()
    assert np.array_equal(s1, s2)
    u1, v1 = kept["u"].cpu().numpy(), kept["v"].cpu().numpy()
    u2, v2 = replay["u"].cpu().numpy(), replay["v"].cpu().numpy()
    # the same terms in the same order; only the contraction of a multiply-add may differ
    du = np.abs(u1 - u2).max()
    dv = np.abs(v1 - v2).max()
    print("kept vs replay: max |du| %.3e, max |dv| %.3e" % (du, dv), flush=True)
    assert du < 1e-12 and dv < 1e-12
    # each pair is a singular pair of zI - A to the working accuracy (backward error)
    nA = np.linalg.norm(A)
    for p in range(len(z)):
        assert abs(np.linalg.norm(v1[p]) - 1) < 1e-10 and abs(np.linalg.norm(u1[p]) - 1) < 1e-10
        res = np.linalg.norm(z[p] * v1[p] - A @ v1[p] - s1[p] * u1[p])
        assert res <= 1e-8 * nA + 1e-6 * s1[p], (p, res)
