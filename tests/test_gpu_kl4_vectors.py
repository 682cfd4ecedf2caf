"""GPU parity of the kernels with singular vectors at kl = 4, the band shapes whose sweeps are
compiled as separate functions (inlined, one of their builds returned wrong sigma on the
Golub-Kahan path): every ku = 0..4, three seeds and three ragged sizes each, with shifts next
to eigenvalues (sigma tiny: the Golub-Kahan path) and across the Gershgorin box (the
bisection, then inverse iteration).  sigma against the oracle to the parity bar, and each
singular pair's residual against the matrix."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import need_gpu, report, tol

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ku", [0, 1, 2, 3, 4])
def test_kl4_vectors_match_oracle(ku):
    torch = need_gpu()
    from paper_2605_04550_amd import api
    kl = 4
    for rep, n in enumerate((97, 150, 203)):
        band = W.random_banded(n, kl, ku, seed=1500 + 10 * ku + rep)
        A = W.to_dense(band)
        lam = np.linalg.eigvals(A)
        rng = np.random.default_rng(1600 + 10 * ku + rep)
        near = lam[rng.choice(n, 12, replace=False)] + 10.0 ** rng.uniform(-7, -3, 12) * np.exp(
            2j * np.pi * rng.uniform(0, 1, 12))
        a, b, c, d = W.gershgorin_box(band)
        far = rng.uniform(a, b, 8) + 1j * rng.uniform(c, d, 8)
        z = np.concatenate([near, far])
        print("kl=4 ku=%d n=%d" % (ku, n), flush=True)
        ref = oracle.sigma_min(band, z)["sigma"]
        mat = api.BandedMatrix.from_band(band)
        r = api.sigma_min(mat, torch.tensor(z, dtype=torch.complex128, device="cuda"), want_vectors=True)
        s = r["sigma"].cpu().numpy()
        info = r["info"].cpu().numpy()
        bnd = tol(band.fro, ref)
        report("kl=4 ku=%d n=%d vectors" % (ku, n), s, ref, bnd)
        assert np.all((info & 2) == 0)
        assert np.all(np.abs(s - ref) <= bnd), np.flatnonzero(np.abs(s - ref) > bnd).tolist()
        assert np.sum((info & 8) == 0) >= 6      # the Golub-Kahan path is exercised
        u, v = r["u"].cpu().numpy(), r["v"].cpu().numpy()
        nA = np.linalg.norm(A)
        for p in range(len(z)):
            assert abs(np.linalg.norm(u[p]) - 1) < 1e-10 and abs(np.linalg.norm(v[p]) - 1) < 1e-10, p
            res = np.linalg.norm(z[p] * v[p] - A @ v[p] - s[p] * u[p])
            assert res <= 1e-8 * nA + 1e-6 * s[p], (p, res)
