"""GPU parity over every compiled band shape: kl, ku in 0..4 (25 kernels per mode).

For each shape a random banded matrix (n = 60 + 7 (5 kl + ku), so the sizes are ragged
against the 8-row chunks) and 16 seeded shifts in its Gershgorin box, from near the
spectrum to the box edge.  Every evaluation mode is compared with the oracle to the parity
bar |sigma - sigma_oracle| <= 1e-10 ||A||_F + 1e-8 sigma_oracle:
  the Golub-Kahan path alone (bisection off), the default (inertia bisection where it
  applies), the vector kernel (sigma, and the residual of the singular pair), and the batch
  kernel on a 4 x 4 grid with and without bisection.
The shapes share one source but are 75 separately compiled kernels (plus 25 batch
kernels), so this is also the check that each compiled kernel computes what the source
says."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import need_gpu, tol

pytestmark = pytest.mark.gpu

SHAPES = [(kl, ku) for kl in range(5) for ku in range(5)]


def _case(kl, ku):
    n = 60 + 7 * (kl * 5 + ku)
    band = W.random_banded(n, kl, ku, seed=1200 + kl * 5 + ku)
    rng = np.random.default_rng(1300 + kl * 5 + ku)
    a, b, c, d = W.gershgorin_box(band)
    z = 0.5 * (a + b) + 0.5j * (c + d) + rng.uniform(0.05, 1.0, 16) * max(b - a, d - c) * np.exp(
        2j * np.pi * rng.uniform(0, 1, 16))
    return band, z, W.Grid(a, b, c, d, 4, 4)


@pytest.mark.parametrize("kl,ku", SHAPES)
def test_every_mode_matches_oracle(kl, ku):
    need_gpu()
    import torch
    from paper_2605_04550_amd import api
    band, z, grid = _case(kl, ku)
    print("shape kl=%d ku=%d n=%d" % (kl, ku, band.n), flush=True)
    ref = oracle.sigma_min(band, z)["sigma"]
    bnd = tol(band.fro, ref)
    mat = api.BandedMatrix.from_band(band)
    zt = torch.tensor(z, dtype=torch.complex128, device="cuda")
    used_bisection = 0
    for tag, kw in (("golub-kahan", dict(bisect=False)), ("default", {}), ("vectors", dict(want_vectors=True))):
        r = api.sigma_min(mat, zt, **kw)
        s = r["sigma"].cpu().numpy()
        info = r["info"].cpu().numpy()
        err = np.abs(s - ref)
        assert np.all(err <= bnd), (tag, kl, ku, np.flatnonzero(err > bnd).tolist(), (err / bnd).max())
        assert np.all((info & 2) == 0), tag
        if tag == "default":
            used_bisection = int(np.sum((info & 8) != 0))
        elif tag == "golub-kahan":
            assert not np.any(info & 8), tag
        else:
            # the singular pair: unit vectors with (zI - A) v = sigma u to the accuracy of sigma
            A = W.to_dense(band)
            u, v = r["u"].cpu().numpy(), r["v"].cpu().numpy()
            for p in range(len(z)):
                res = np.linalg.norm((z[p] * np.eye(band.n) - A) @ v[p] - s[p] * u[p])
                assert abs(np.linalg.norm(u[p]) - 1) < 1e-12 and abs(np.linalg.norm(v[p]) - 1) < 1e-12
                assert res <= 4 * bnd[p] + 1e-12 * band.fro, (kl, ku, p, res, bnd[p])
    if kl + ku >= 1:
        assert used_bisection >= 8         # the far half of the shifts qualifies
    refg = oracle.sigma_min(band, oracle.grid_points(grid))["sigma"]
    for bis in (False, True):
        rb = api.BandedBatch([mat], [grid]).eval(None, bisect=bis)
        s = rb["sigma"].cpu().numpy()
        assert np.all(np.abs(s - refg) <= tol(band.fro, refg)), ("batch", bis)
