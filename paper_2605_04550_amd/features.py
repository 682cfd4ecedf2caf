"""Matrix features of Sec. 3.1 for the mask producer: the 30 global features f1 .. f30 (Tables
matrix, matrixAdd and resolvent) and the spectrum, computed once per matrix on the host.

These are per-matrix dense linear algebra (eigenvalues, eigenvectors, singular values of an
n = 64 matrix): input preparation for the classifier, not data-parallel work over the grid.
Readings where the paper is not explicit:
  * features are taken from A itself, with the normalisations the tables write out (f11, f12,
    f14 .. f16 by ||A||_F; f22, f23 on A~ = A / (||A||_F + 1e-12));
  * std is the population standard deviation; epsilon = delta = 1e-12 wherever the tables add
    one for numerical safety;
  * kappa(V) is the 2-norm condition number of the eigenvector matrix with unit columns;
  * f28 .. f30: one standard normal right-hand side b per matrix (seeded by the caller) for the
    three shifts z_delta = (mean of the eigenvalues) + delta, delta = 0.5, 1, 2.
"""
from __future__ import annotations

import numpy as np

EPS = 1e-12


def dense_from_band(ab, n, kl, ku):
    """The dense matrix of a LAPACK general-band array ab[j, ku + i - j] = A[i, j]."""
    A = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            A[i, j] = ab[j, ku + i - j]
    return A


def global_features(A, seed: int = 0):
    """(f [30] float64, eigenvalues [n] complex128) of the n x n matrix A (Sec. 3.1)."""
    A = np.asarray(A)
    A = A.astype(np.complex128) if np.iscomplexobj(A) else A.astype(np.float64)
    n = A.shape[0]
    fro = np.linalg.norm(A)
    lam, V = np.linalg.eig(A)
    s = np.linalg.svd(A, compute_uv=False)
    re, im, ab = lam.real, lam.imag, np.abs(lam)
    f = np.empty(30)
    f[0], f[1], f[2], f[3] = re.mean(), re.std(), re.min(), re.max()
    f[4], f[5], f[6], f[7] = im.mean(), im.std(), im.min(), im.max()
    f[8], f[9] = ab.max(), ab.min()
    f[10] = np.linalg.norm(A - A.T) / fro
    f[11] = np.linalg.norm(A - A.conj().T) / fro
    f[12] = np.log10(s[0] / s[-1] + EPS) if s[-1] > 0 else np.log10(1e300)
    f[13] = s[0] / fro
    f[14] = np.abs(A).sum(axis=0).max() / fro
    f[15] = np.abs(A).sum(axis=1).max() / fro
    d = np.abs(np.diag(A))
    off = np.abs(A - np.diag(np.diag(A)))
    f[16], f[17] = d.mean(), d.std()
    f[18], f[19] = off.mean(), off.std()
    f[20] = np.count_nonzero(np.abs(A) > 1e-10) / float(n * n)
    at2 = np.abs(A / (fro + EPS)) ** 2
    f[21], f[22] = at2.mean(), at2.std()
    sv = np.linalg.svd(V, compute_uv=False)
    f[23] = np.log10(sv[0] / sv[-1] + EPS) if sv[-1] > 0 else np.log10(1e300)
    f[24] = np.log10(np.linalg.norm(A - A.conj().T) / fro + EPS)
    f[25] = (s[0] - s[-1]) / (s[0] + EPS)
    f[26] = (ab.max() - ab.min()) / (ab.max() + EPS)
    b = np.random.default_rng(seed).standard_normal(n)
    cent = lam.mean()
    for k, delta in enumerate((0.5, 1.0, 2.0)):
        try:
            x = np.linalg.solve((cent + delta) * np.eye(n) - A, b.astype(np.complex128))
            f[27 + k] = np.log10(np.linalg.norm(x) / np.linalg.norm(b))
        except np.linalg.LinAlgError:            # z_delta exactly an eigenvalue: the resolvent is unbounded
            f[27 + k] = 16.0
    return f, lam


def band_features(band, seed: int = 0):
    """global_features of a band (an object with ab, n, kl, ku)."""
    A = dense_from_band(band.ab, band.n, band.kl, band.ku)
    if getattr(band, "real", False):
        A = A.real
    return global_features(A, seed)
