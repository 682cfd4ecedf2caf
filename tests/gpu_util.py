"""Helpers shared by the GPU tests (no arithmetic of the method lives here)."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_04550_amd as P
    P.lib()          # raises if the HIP library is missing: no fallback
    return torch


def tol(fro, sigma_ref, tol_norm=1e-10, tol_rel=1e-8):
    """Parity bar: |sigma_gpu - sigma_oracle| <= tol_norm * ||A||_F + tol_rel * sigma_oracle."""
    return tol_norm * fro + tol_rel * np.asarray(sigma_ref)


def golden(name):
    path = os.path.join(GOLDEN, name + ".npz")
    if not os.path.exists(path):
        pytest.skip("golden set %s not generated" % name)
    return dict(np.load(path, allow_pickle=False))


def report(name, sig_gpu, sig_ref, bound):
    err = np.abs(sig_gpu - sig_ref)
    worst = int(np.argmax(err / bound))
    print("%s: %d points, max |err| %.3e, max err/bound %.3e (at %d: gpu %.17g ref %.17g)"
          % (name, len(err), err.max(), (err / bound).max(), worst, sig_gpu[worst], sig_ref[worst]), flush=True)
