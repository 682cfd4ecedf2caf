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


def offdiag_sums(band):
    """Row and column sums of |a_ij| over i != j (GB layout: ab[j, ku + i - j] = A[i, j])."""
    n, kl, ku = band.n, band.kl, band.ku
    r = np.zeros(n)
    c = np.zeros(n)
    for d in range(kl + ku + 1):
        off = d - ku                      # i - j
        if off == 0:
            continue
        j = np.arange(max(0, -off), min(n, n - off))
        a = np.abs(band.ab[j, d])
        np.add.at(r, j + off, a)
        np.add.at(c, j, a)
    return r, c


def johnson_bound(band, z):
    """Johnson (1989): sigma_min(zI - A) >= min_i (|z - a_ii| - (r_i + c_i) / 2)."""
    r, c = offdiag_sums(band)
    half = 0.5 * (r + c)
    dg = band.ab[:, band.ku]
    return np.array([np.min(np.abs(zz - dg) - half) for zz in np.atleast_1d(z)])


def column_norm_bound(band, z):
    """sigma_min(zI - A) <= min_j |(zI - A) e_j| (the smallest column norm)."""
    n, kl, ku = band.n, band.kl, band.ku
    out = []
    for zz in np.atleast_1d(z):
        col2 = np.zeros(n)
        for d in range(kl + ku + 1):
            off = d - ku                  # i - j
            j = np.arange(max(0, -off), min(n, n - off))
            v = -band.ab[j, d] + (zz if off == 0 else 0.0)
            np.add.at(col2, j, np.abs(v) ** 2)
        out.append(np.sqrt(col2.min()))
    return np.array(out)


def certify(band, z, sigma, delta, name):
    """Both sides by the oracle's inertia count: no singular value of zI - A below sigma - delta,
    at least one below sigma + delta.  Callers keep sigma well above zero (the count factorises
    [[-t I, M], [M^H, -t I]] without pivoting)."""
    import oracle
    lo = oracle.count_below(band, z, sigma - delta)
    hi = oracle.count_below(band, z, sigma + delta)
    bad = np.flatnonzero((lo != 0) | (hi < 1))
    print("%s: inertia certificate on %d points, %d failures" % (name, len(z), len(bad)), flush=True)
    assert len(bad) == 0, [(int(p), z[p], sigma[p], int(lo[p]), int(hi[p])) for p in bad[:5]]
