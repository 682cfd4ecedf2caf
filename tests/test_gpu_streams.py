"""GPU test: calls on several streams sharing one matrix handle.  Each caller stream gets its own
side stream for the Golub-Kahan launch (up to four; further streams share the first), so the
calls overlap; every result must equal the same call made alone on the default stream, bit for
bit (a shift's arithmetic does not depend on which lane or launch takes it)."""
import numpy as np
import pytest

import workloads as W
from gpu_util import need_gpu

pytestmark = pytest.mark.gpu


def test_concurrent_calls_on_one_handle_equal_serial_calls():
    need_gpu()
    import torch
    from paper_2605_04550_amd import api
    # tridiagonal Toeplitz: inside the ellipse sigma_min is tiny (the Golub-Kahan path), outside
    # it the bisection takes the shifts, so every call uses both kernels
    band = W.toeplitz(600, 0.25, 0.0, 1.0)
    mat = api.BandedMatrix.from_band(band)
    grid = W.Grid(-2.0, 2.0, -2.0, 2.0, 96, 80)
    rng = np.random.default_rng(515)
    masks = [torch.tensor((rng.uniform(size=(grid.ny, grid.nx)) < f).astype(np.uint8), device="cuda")
             for f in (0.3, 0.5, 0.7, 0.4, 0.6)]

    def call(mask, stream=None):
        if mask is None:
            return api.eval_grid(mat, grid, eps=1e-2, stream=stream)
        return api.eval_grid(mat, grid, mask, eps=1e-2, stream=stream)

    work = [None] + masks                       # six calls: more streams than side streams
    ref = [call(m) for m in work]
    torch.cuda.synchronize()
    gk = [int((r["iters"].cpu().numpy() > 0).sum()) for r in ref]
    print("serial: Golub-Kahan shifts per call %s" % gk, flush=True)
    assert min(gk) > 0
    streams = [torch.cuda.Stream() for _ in work]
    for rep in range(3):
        out = []
        for m, s in zip(work, streams):
            with torch.cuda.stream(s):
                out.append(call(m, stream=s))
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(ref, out)):
            cnt = int(a["count"].item())
            assert int(b["count"].item()) == cnt, (rep, k)
            for key in ("idx", "sigma", "info", "iters", "sens"):
                assert torch.equal(a[key][:cnt], b[key][:cnt]), (rep, k, key)
    print("3 rounds of %d concurrent calls equal the serial ones" % len(work), flush=True)
    # the same calls from two host threads at once (ctypes calls release the interpreter lock,
    # so the enqueue sequences of calls sharing a side stream can interleave)
    import threading
    for rep in range(3):
        out = [None] * len(work)

        def run(ks):
            for k in ks:
                with torch.cuda.stream(streams[k]):
                    out[k] = call(work[k], stream=streams[k])

        th = [threading.Thread(target=run, args=(range(j, len(work), 2),)) for j in range(2)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(ref, out)):
            cnt = int(a["count"].item())
            assert int(b["count"].item()) == cnt, (rep, k)
            for key in ("idx", "sigma", "info", "iters", "sens"):
                assert torch.equal(a[key][:cnt], b[key][:cnt]), (rep, k, key)
    print("3 rounds of the calls from two threads equal the serial ones", flush=True)
