"""GPU test of ps_eval_points_noalloc, the allocation-free form of ps_eval_points (sigma only,
the library's fixed device scratch as workspace): two calls in a row, the second with fewer
shifts, each against ps_eval_points on the same shifts, through the C ABI."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import need_gpu, tol

pytestmark = pytest.mark.gpu


def _cases():
    g = W.Grid(-1.5, 3.0, -3.5, 3.5, 64, 64)
    rb = W.random_banded(3000, 2, 3, seed=9)
    a, b, c, d = W.gershgorin_box(rb)
    return [(W.grcar(100), oracle.grid_points(g)),
            (rb, oracle.grid_points(W.Grid(a, b, c, d, 48, 48)))]


def test_noalloc_matches_eval_points_on_two_calls():
    need_gpu()
    import torch
    from paper_2605_04550_amd import api, ps_eval_points_noalloc
    for band, zs in _cases():
        mat = api.BandedMatrix.from_band(band)
        for npts in (len(zs), len(zs) // 3 + 1):          # the second call is smaller
            print("noalloc: n=%d kl=%d ku=%d npts=%d" % (band.n, band.kl, band.ku, npts), flush=True)
            z = torch.tensor(zs[:npts], dtype=torch.complex128, device="cuda")
            sig = torch.full((npts,), float("nan"), dtype=torch.float64, device="cuda")
            info = torch.full((npts,), -1, dtype=torch.int32, device="cuda")
            o = api.make_opts()
            stream = torch.cuda.current_stream().cuda_stream
            ps_eval_points_noalloc(mat.handle, z.data_ptr(), npts, o, sig.data_ptr(), info.data_ptr(), 0, stream)
            ref = api.sigma_min(mat, z)
            torch.cuda.synchronize()
            s1, s0 = sig.cpu().numpy(), ref["sigma"].cpu().numpy()
            i1, i0 = info.cpu().numpy(), ref["info"].cpu().numpy()
            assert np.all(np.isfinite(s1))
            bound = tol(band.fro, s0)
            assert np.all(np.abs(s1 - s0) <= bound), np.max(np.abs(s1 - s0) / bound)
            # the same kernels on the same shifts: the same outcome per shift
            assert np.array_equal(i1 & 0xff, i0 & 0xff)
            print("noalloc: max |diff| / bound %.3g, identical %s" % (np.max(np.abs(s1 - s0) / bound),
                                                                     np.array_equal(s1, s0)), flush=True)


def test_noalloc_refuses_what_does_not_fit_and_vectors():
    need_gpu()
    import torch
    from paper_2605_04550_amd import PsError, api, ps_eval_points_noalloc
    band = W.random_banded(20000, 4, 4, seed=3)
    mat = api.BandedMatrix.from_band(band)
    z = torch.zeros(1, dtype=torch.complex128, device="cuda")
    sig = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(PsError) as e:
        ps_eval_points_noalloc(mat.handle, z.data_ptr(), 1, api.make_opts(), sig.data_ptr())
    assert "WORKSPACE" in str(e.value) and "scratch" in str(e.value)
    small = api.BandedMatrix.from_band(W.grcar(50))
    with pytest.raises(PsError) as e:
        ps_eval_points_noalloc(small.handle, z.data_ptr(), 1, api.make_opts(want_vectors=True), sig.data_ptr())
    assert "UNSUPPORTED" in str(e.value)
