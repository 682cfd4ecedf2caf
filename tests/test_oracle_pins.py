"""Pins for the CPU oracle: closed forms, invariants, brute force and the paper's example.

Each pin is independent of the oracle's own code: closed forms of normal matrices
(Sec. 2, resolvent-norm definition: sigma_min(zI - A) = dist(z, spectrum) for normal A),
the 2 x 2 closed form, brute force on 3 x 3 characteristic polynomials, LAPACK as a third
opinion, and invariants that hold for every matrix.  ``test_oracle_mutants`` plants
mistakes in a copy of the oracle's C source and checks that these pins catch each one.
"""
import ctypes
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EPS = 2.0 ** -53


def _tol(band, sigma=0.0):
    """Oracle accuracy target for pins: a small multiple of n * eps * ||M||."""
    return 64 * band.n * EPS * (band.fro + 4.0) + 1e-13 * sigma


def _rng(k):
    return np.random.default_rng(1000 + k)


# ----------------------------------------------------------------------------- closed forms

def test_n1_closed_form():
    rng = _rng(1)
    for _ in range(20):
        a = complex(*rng.standard_normal(2))
        band = W.diagonal([a])
        z = rng.standard_normal(5) + 1j * rng.standard_normal(5)
        s = oracle.sigma_min(band, z)["sigma"]
        np.testing.assert_allclose(s, np.abs(z - a), rtol=1e-15, atol=1e-15)


def test_2x2_closed_form():
    # sigma_min = |det M| / sigma_max, sigma_max^2 = (|M|_F^2 + sqrt(|M|_F^4 - 4 |det M|^2)) / 2
    rng = _rng(2)
    for _ in range(50):
        A = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
        ab = np.zeros((2, 3), dtype=complex)
        for j in range(2):
            for i in range(2):
                ab[j, 1 + i - j] = A[i, j]
        band = W.Band(ab, 2, 1, 1)
        z = complex(*rng.standard_normal(2))
        M = z * np.eye(2) - A
        det = abs(M[0, 0] * M[1, 1] - M[0, 1] * M[1, 0])
        f2 = float(np.sum(np.abs(M) ** 2))
        smax = math.sqrt((f2 + math.sqrt(max(f2 * f2 - 4 * det * det, 0.0))) / 2)
        s = oracle.sigma_min(band, [z])["sigma"][0]
        assert abs(s - det / smax) <= 1e-14 * smax


def test_diagonal_distance():
    rng = _rng(3)
    vals = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    band = W.diagonal(vals)
    z = rng.standard_normal(64) * 2 + 2j * rng.standard_normal(64)
    s = oracle.sigma_min(band, z)["sigma"]
    ref = np.min(np.abs(z[:, None] - vals[None, :]), axis=1)
    np.testing.assert_allclose(s, ref, rtol=0, atol=1e-14)
    # z on an eigenvalue: exactly singular
    s0 = oracle.sigma_min(band, vals[:3])["sigma"]
    assert np.all(s0 == 0.0)


@pytest.mark.parametrize("n,a,b", [(30, 0.3, 0.7 + 0.2j), (57, -1.0, 1.5j), (64, 0.0, 1.0)])
def test_hermitian_tridiagonal_toeplitz(n, a, b):
    band = W.hermitian_toeplitz_tridiag(n, a, b)
    lam = a + 2 * abs(b) * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    rng = _rng(4)
    z = rng.uniform(-4, 4, 40) + 1j * rng.uniform(-2, 2, 40)
    s = oracle.sigma_min(band, z)["sigma"]
    ref = np.min(np.abs(z[:, None] - lam[None, :]), axis=1)
    np.testing.assert_allclose(s, ref, rtol=0, atol=_tol(band))


def test_polynomial_of_hermitian_is_normal_banded():
    n = 48
    coeffs = [0.2 - 0.1j, 1.0 + 0.5j, 0.3j, -0.25, 0.05 + 0.05j]     # degree 4: kl = ku = 4
    band = W.band_poly_hermitian(n, 0.1, 0.6 + 0.3j, coeffs)
    lamH = 0.1 + 2 * abs(0.6 + 0.3j) * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    lam = sum(c * lamH ** k for k, c in enumerate(coeffs))
    rng = _rng(5)
    z = rng.uniform(-2, 2, 40) + 1j * rng.uniform(-2, 2, 40)
    s = oracle.sigma_min(band, z)["sigma"]
    ref = np.min(np.abs(z[:, None] - lam[None, :]), axis=1)
    np.testing.assert_allclose(s, ref, rtol=0, atol=_tol(band))
    # rotated and shifted: e^{i theta} H + c I
    th, cc = 0.7, 0.3 - 0.2j
    bandr = W.band_from_rows(n, 1, 1, {-1: np.exp(1j * th) * np.conj(0.6 + 0.3j),
                                       0: np.exp(1j * th) * 0.1 + cc,
                                       1: np.exp(1j * th) * (0.6 + 0.3j)})
    lamr = np.exp(1j * th) * lamH + cc
    s = oracle.sigma_min(bandr, z)["sigma"]
    np.testing.assert_allclose(s, np.min(np.abs(z[:, None] - lamr[None, :]), axis=1), atol=_tol(bandr))


@pytest.mark.parametrize("n", [5, 9, 16])
def test_circulant_full_band(n):
    rng = _rng(6 + n)
    col0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    band = W.circulant_full(col0)
    lam = np.fft.fft(col0)          # eigenvalues of C[i,j] = c[(i-j) mod n]
    z = rng.standard_normal(30) * 3 + 3j * rng.standard_normal(30)
    s = oracle.sigma_min(band, z)["sigma"]
    ref = np.min(np.abs(z[:, None] - lam[None, :]), axis=1)
    np.testing.assert_allclose(s, ref, rtol=0, atol=_tol(band))


def _read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_paper_jordan_example():
    g = _read_golden("jordan32.txt")
    n, delta = int(g["n"]), g["delta"]
    A = W.jordan(n)
    s0 = oracle.sigma_min(A, [0.0])["sigma"][0]
    assert s0 == g["sigma_min_A_at_0"]
    B = W.jordan_perturbed(n, delta)
    lam = g["eigenvalue_modulus"] * np.exp(2j * np.pi * np.arange(n) / n)
    s = oracle.sigma_min(B, lam)["sigma"]
    assert np.all(s <= 1e-13), s.max()
    # off the circle the matrix is far from singular
    s_off = oracle.sigma_min(B, 0.5 * lam[:4])["sigma"]
    assert np.all(s_off > 1e-6)


# ----------------------------------------------------------------------------- brute force / third opinion

def _charpoly_smallest_root_3x3(M):
    """Smallest eigenvalue of G = M^H M (3 x 3) from its characteristic polynomial, by bisection."""
    G = M.conj().T @ M
    c2 = -np.trace(G).real
    c1 = (G[0, 0] * G[1, 1] - G[0, 1] * G[1, 0] + G[0, 0] * G[2, 2] - G[0, 2] * G[2, 0]
          + G[1, 1] * G[2, 2] - G[1, 2] * G[2, 1]).real
    c0 = -(G[0, 0] * (G[1, 1] * G[2, 2] - G[1, 2] * G[2, 1])
           - G[0, 1] * (G[1, 0] * G[2, 2] - G[1, 2] * G[2, 0])
           + G[0, 2] * (G[1, 0] * G[2, 1] - G[1, 1] * G[2, 0])).real
    p = lambda t: ((t + c2) * t + c1) * t + c0
    # p(t) = det(tI - G) is negative below the smallest root; scan [0, min diag G]
    # (lambda_min <= min diagonal entry) for the first sign change, then bisect.
    top = float(np.min(np.diag(G).real))
    ts = np.linspace(0.0, top, 20001)
    k = int(np.argmax(p(ts) >= 0))
    lo, hi = (ts[k - 1], ts[k]) if k > 0 else (0.0, 0.0)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if p(mid) < 0:      # p(0) = -det(G) <= 0 and p < 0 below the smallest root
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def test_brute_force_3x3():
    rng = _rng(7)
    for _ in range(40):
        A = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        ab = np.zeros((3, 5), dtype=complex)
        for j in range(3):
            for i in range(3):
                ab[j, 2 + i - j] = A[i, j]
        band = W.Band(ab, 3, 2, 2)
        z = complex(*rng.standard_normal(2))
        t = _charpoly_smallest_root_3x3(z * np.eye(3) - A)
        s = oracle.sigma_min(band, [z])["sigma"][0]
        assert abs(s * s - t) <= 1e-11 * (1 + np.sum(np.abs(A) ** 2)), (s * s, t)


def test_lapack_third_opinion_random_banded():
    rng = _rng(8)
    for kl, ku in [(0, 1), (1, 0), (2, 3), (4, 1), (3, 3)]:
        band = W.random_banded(37, kl, ku, seed=int(rng.integers(1 << 30)))
        A = W.to_dense(band)
        z = rng.standard_normal(8) + 1j * rng.standard_normal(8)
        r = oracle.sigma_min(band, z, all_sv=True)
        for k, zz in enumerate(z):
            sv = np.linalg.svd(zz * np.eye(37) - A, compute_uv=False)
            assert abs(r["sigma"][k] - sv[-1]) <= _tol(band)
            np.testing.assert_allclose(np.sort(r["sall"][k])[::-1], sv, atol=_tol(band))


# ----------------------------------------------------------------------------- invariants

def test_invariants_grcar_grid():
    band = W.grcar(60)
    grid = W.Grid(-1.5, 3.0, -3.5, 3.5, 24, 24)
    z = oracle.grid_points(grid)
    s = oracle.sigma_min(band, z)["sigma"]
    tol = _tol(band)
    # 1-Lipschitz in z (Weyl): neighbours along rows and columns
    S = s.reshape(grid.ny, grid.nx)
    Z = z.reshape(grid.ny, grid.nx)
    assert np.all(np.abs(np.diff(S, axis=1)) <= np.abs(np.diff(Z, axis=1)) + tol)
    assert np.all(np.abs(np.diff(S, axis=0)) <= np.abs(np.diff(Z, axis=0)) + tol)
    # real A: sigma(conj z) = sigma(z); this grid is symmetric about the real axis
    np.testing.assert_allclose(S, S[::-1, :], atol=tol)
    # sigma <= dist(z, spectrum) (eigenvalues by LAPACK, within its own error)
    lam = np.linalg.eigvals(W.to_dense(band))
    dist = np.min(np.abs(z[:, None] - lam[None, :]), axis=1)
    assert np.all(s <= dist + 1e-8)


def test_invariants_transpose_similarity_scaling():
    rng = _rng(9)
    band = W.random_banded(41, 2, 3, seed=77)
    A = W.to_dense(band)
    z = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    s = oracle.sigma_min(band, z)["sigma"]
    tol = _tol(band)
    # sigma(zI - A) = sigma(zI - A^T) (kl and ku swap)
    At = A.T
    abt = np.zeros((41, 6), dtype=complex)
    for j in range(41):
        for i in range(max(0, j - 2), min(41, j + 4)):
            abt[j, 2 + i - j] = At[i, j]
    st = oracle.sigma_min(W.Band(abt, 41, 3, 2), z)["sigma"]
    np.testing.assert_allclose(st, s, atol=tol)
    # unitary diagonal similarity D A D^H
    d = np.exp(1j * rng.uniform(0, 2 * np.pi, 41))
    Ad = (d[:, None] * A) * np.conj(d)[None, :]
    abd = np.zeros_like(band.ab)
    for j in range(41):
        for i in range(max(0, j - 3), min(41, j + 3)):
            abd[j, 3 + i - j] = Ad[i, j]
    sd = oracle.sigma_min(W.Band(abd, 41, 2, 3), z)["sigma"]
    np.testing.assert_allclose(sd, s, atol=tol)
    # scaling: sigma(alpha z I - alpha A) = |alpha| sigma(zI - A)
    alpha = 1.7 - 0.4j
    ss = oracle.sigma_min(W.Band(band.ab * alpha, 41, 2, 3), z * alpha)["sigma"]
    np.testing.assert_allclose(ss, abs(alpha) * s, atol=abs(alpha) * tol)
    # Johnson (1989) lower bound: sigma_min(M) >= min_i (|m_ii| - (r_i + c_i)/2)
    for k, zz in enumerate(z):
        M = zz * np.eye(41) - A
        absM = np.abs(M)
        off = absM - np.diag(np.diag(absM))
        lb = np.min(np.abs(np.diag(M)) - 0.5 * (off.sum(axis=1) + off.sum(axis=0)))
        assert s[k] >= lb - tol


def test_toeplitz_exact_spectrum_bound():
    # Tridiagonal Toeplitz (sub c, diag a, super b): eigenvalues a + 2 sqrt(b c) cos(k pi/(n+1))
    n = 120
    band = W.toeplitz(n, 0.25, 0.0, 1.0)
    lam = 2 * math.sqrt(0.25) * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    rng = _rng(10)
    z = rng.uniform(-2, 2, 40) + 1j * rng.uniform(-2, 2, 40)
    s = oracle.sigma_min(band, z)["sigma"]
    dist = np.min(np.abs(z[:, None] - lam[None, :]), axis=1)
    assert np.all(s <= dist + _tol(band))


# ----------------------------------------------------------------------------- vectors, grid, mask, adjoint, Newton

def test_singular_vectors_residual_and_phase():
    band = W.grcar(50)
    A = W.to_dense(band)
    z = np.array([0.5 + 1.0j, 2.0 - 0.3j, -1.0 + 2.0j])
    r = oracle.sigma_min(band, z, want_vectors=True)
    for k, zz in enumerate(z):
        M = zz * np.eye(50) - A
        u, v, s = r["u"][k], r["v"][k], r["sigma"][k]
        assert abs(np.linalg.norm(u) - 1) < 1e-13 and abs(np.linalg.norm(v) - 1) < 1e-13
        assert np.linalg.norm(M @ v - s * u) <= 1e-12 * np.linalg.norm(M)
        assert np.linalg.norm(M.conj().T @ u - s * v) <= 1e-12 * np.linalg.norm(M)
        kmax = int(np.argmax(np.abs(v)))
        assert abs(v[kmax].imag) < 1e-15 and v[kmax].real > 0


def test_lapack_pair_closed_form_and_jacobi():
    """smallest_pair_lapack (used for the n = 4000 gradients): the distance to the nearest and
    second-nearest eigenvalue of a diagonal matrix with the matching unit vectors; residuals
    M v = sigma u, M^H u = sigma v; the Jacobi oracle's sigma_n, sigma_{n-1} and adjoint at n = 60."""
    lam = np.array([0.5, -1.0 + 1.0j, 2.0j, 1.5 - 0.5j, -0.3])
    z = np.array([0.4 + 0.1j, 1.0 - 0.2j, -0.5 + 1.7j])
    r = oracle.smallest_pair_lapack(W.diagonal(lam), z)
    d = np.abs(z[:, None] - lam[None, :])
    np.testing.assert_allclose(r["sigma"], np.sort(d, axis=1)[:, 0], rtol=1e-15)
    np.testing.assert_allclose(r["s2"], np.sort(d, axis=1)[:, 1], rtol=1e-15)
    for p in range(3):
        k = int(np.argmin(d[p]))
        assert abs(abs(r["v"][p, k]) - 1) < 1e-15 and abs(abs(r["u"][p, k]) - 1) < 1e-15
        np.testing.assert_allclose(r["u"][p, k], r["v"][p, k] * (z[p] - lam[k]) / d[p, k], atol=1e-15)
    for band in (W.grcar(60), W.random_banded(60, 2, 1, seed=8)):
        A = W.to_dense(band)
        zz = np.array([0.7 + 1.2j, 2.1 - 0.4j, -0.2 + 0.1j])
        a = oracle.smallest_pair_lapack(band, zz)
        j = oracle.sigma_min(band, zz, want_vectors=True, all_sv=True)
        s = np.sort(j["sall"], axis=1)
        nm = np.linalg.norm(A) + 3
        np.testing.assert_allclose(a["sigma"], s[:, 0], atol=1e-13 * nm)
        np.testing.assert_allclose(a["s2"], s[:, 1], atol=1e-13 * nm)
        for p in range(3):
            M = zz[p] * np.eye(60) - A
            assert np.linalg.norm(M @ a["v"][p] - a["sigma"][p] * a["u"][p]) <= 1e-13 * nm
            assert np.linalg.norm(M.conj().T @ a["u"][p] - a["sigma"][p] * a["v"][p]) <= 1e-13 * nm
        w = np.array([1.0, -0.5, 2.0])
        ga = oracle.adjoint(band, a["u"], a["v"], w)
        gj = oracle.adjoint(band, j["u"], j["v"], w)
        np.testing.assert_allclose(ga[0], gj[0], atol=1e-10)
        np.testing.assert_allclose(ga[1], gj[1], atol=1e-10)


def test_grid_points_definition():
    g = W.Grid(-1.0, 3.0, -2.0, 2.0, 5, 3)
    z = oracle.grid_points(g).reshape(3, 5)
    assert z[0, 0] == complex(-1, -2) and z[2, 4] == complex(3, 2)
    np.testing.assert_allclose(np.diff(z.real, axis=1), 1.0)
    np.testing.assert_allclose(np.diff(z.imag, axis=0), 2.0)
    z1 = oracle.grid_points(W.Grid(0.5, 9.0, 1.5, 9.0, 1, 1))
    assert z1[0] == complex(0.5, 1.5)


def test_compact_mask_and_sensitive():
    m = np.zeros((4, 5), dtype=np.uint8)
    m[1, 2] = m[3, 0] = m[0, 4] = 1
    assert list(oracle.compact_mask(m)) == [4, 7, 15]
    assert list(oracle.sensitive([0.5, 0.01, 0.0100001, 0.0], 0.01)) == [0, 1, 0, 1]


def test_adjoint_closed_forms_and_fd():
    # n = 1: d|z - a|/dz = (z - a)/|z - a|, dA = -(same)
    a = 0.3 - 0.2j
    band = W.diagonal([a])
    z = np.array([1.1 + 0.4j, -0.7 - 0.9j])
    r = oracle.sigma_min(band, z, want_vectors=True)
    gz, gb = oracle.adjoint(band, r["u"], r["v"], np.ones(2))
    np.testing.assert_allclose(gz, (z - a) / np.abs(z - a), atol=1e-15)
    np.testing.assert_allclose(gb[0, 0], -np.sum((z - a) / np.abs(z - a)), atol=1e-15)
    # general banded: central differences of the oracle itself
    band = W.random_banded(12, 1, 2, seed=5)
    rng = _rng(11)
    z = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    w = rng.standard_normal(3)
    r = oracle.sigma_min(band, z, want_vectors=True)
    gz, gb = oracle.adjoint(band, r["u"], r["v"], w)
    h = 1e-6
    sp = oracle.sigma_min(band, z + h)["sigma"]
    sm = oracle.sigma_min(band, z - h)["sigma"]
    spi = oracle.sigma_min(band, z + 1j * h)["sigma"]
    smi = oracle.sigma_min(band, z - 1j * h)["sigma"]
    fd = w * ((sp - sm) + 1j * (spi - smi)) / (2 * h)
    np.testing.assert_allclose(gz, fd, atol=1e-7)
    L = lambda ab: float(np.sum(w * oracle.sigma_min(W.Band(ab, 12, 1, 2), z)["sigma"]))
    for (j, rr) in [(3, 0), (5, 1), (7, 2), (10, 3)]:
        for unit in (1.0, 1j):
            abp = band.ab.copy(); abp[j, rr] += unit * h
            abm = band.ab.copy(); abm[j, rr] -= unit * h
            d = (L(abp) - L(abm)) / (2 * h)
            got = gb[j, rr].real if unit == 1.0 else gb[j, rr].imag
            assert abs(got - d) < 1e-7, (j, rr, unit, got, d)


def test_newton_step_circle_contour():
    # diagonal A: the eps-level set near an isolated eigenvalue a is the circle |z - a| = eps
    a = 0.4 + 0.1j
    band = W.diagonal([a, 5.0, -5.0])
    eps = 1e-3
    z = a + np.array([1.3e-3, 0.8e-3j, -1.1e-3 - 0.4e-3j])
    for _ in range(3):
        r = oracle.sigma_min(band, z, want_vectors=True)
        gz, _ = oracle.adjoint(band, r["u"], r["v"], np.ones(len(z)))
        z = oracle.newton_step(z, r["sigma"], gz, eps)
    np.testing.assert_allclose(np.abs(z - a), eps, rtol=1e-6)


# ----------------------------------------------------------------------------- inertia count

def test_count_below_closed_form_diagonal():
    # normal A: the singular values of zI - A are |z - a_k| exactly
    rng = _rng(41)
    vals = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    band = W.diagonal(vals)
    z = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    for zz in z:
        s = np.sort(np.abs(zz - vals))
        ts = np.concatenate([[0.5 * s[0]], 0.5 * (s[:-1] + s[1:]), [2 * s[-1]]])
        got = oracle.count_below(band, np.full(len(ts), zz), ts)
        assert np.array_equal(got, np.arange(len(ts))), (zz, got)


def test_count_below_matches_all_singular_values():
    # general banded matrices: counts at thresholds between consecutive singular values of
    # the dense SVD (all of them, from the Jacobi oracle) and just around sigma_min
    for k, (n, kl, ku) in enumerate([(17, 2, 1), (25, 0, 3), (30, 3, 0), (12, 4, 4), (40, 1, 1)]):
        band = W.random_banded(n, kl, ku, seed=60 + k)
        rng = _rng(50 + k)
        z = rng.uniform(-2, 2, 3) + 1j * rng.uniform(-2, 2, 3)
        r = oracle.sigma_min(band, z, all_sv=True)
        lap = np.linalg.svd(z[:, None, None] * np.eye(n) - W.to_dense(band), compute_uv=False)
        for p in range(len(z)):
            s = np.sort(r["sall"][p])
            np.testing.assert_allclose(s, np.sort(lap[p]), atol=1e-12)
            ts = np.concatenate([[s[0] * (1 - 1e-6), s[0] * (1 + 1e-6)], 0.5 * (s[1:-1] + s[2:])])
            expect = np.concatenate([[0, 1], np.arange(2, n)])
            got = oracle.count_below(band, np.full(len(ts), z[p]), ts)
            assert np.array_equal(got, expect), (n, kl, ku, p, got, expect)


def test_count_below_toeplitz_larger_n():
    # the non-normal tridiagonal Toeplitz matrix at n = 500, away from and near its spectrum:
    # count(sigma_min (1 -/+ 1e-9)) = 0 / >= 1 with sigma_min from the Jacobi oracle
    band = W.toeplitz(500, 0.25, 0.0, 1.0)
    z = np.array([1.9 + 1.9j, -1.7 + 0.2j])
    r = oracle.sigma_min(band, z)
    lo = oracle.count_below(band, z, r["sigma"] * (1 - 1e-9))
    hi = oracle.count_below(band, z, r["sigma"] * (1 + 1e-9))
    assert np.all(lo == 0) and np.all(hi >= 1), (lo, hi)


# ----------------------------------------------------------------------------- contour seeds

def test_contour_seeds_on_a_circle():
    # n = 1, A = [a]: sigma_min(z) = |z - a|, so the eps-level curve is the circle |z - a| = eps
    a = 0.1 - 0.05j
    band = W.diagonal([a])
    grid = W.Grid(-1.0, 1.0, -1.0, 1.0, 81, 61)
    z = oracle.grid_points(grid)
    sigma = np.abs(z - a)
    eps = 0.55
    seeds = oracle.contour_seeds(grid, sigma, eps)
    inside = (sigma <= eps).reshape(61, 81)
    n_edges = np.sum(inside[:, 1:] != inside[:, :-1]) + np.sum(inside[1:, :] != inside[:-1, :])
    assert len(seeds) == n_edges > 0
    # every seed lies on a grid edge crossing the circle, close to the circle (second-order
    # error of the ln-linear interpolation over a spacing of 1/40)
    assert np.all(np.abs(np.abs(seeds - a) - eps) < 2e-3)
    hx, hy = 2.0 / 80, 2.0 / 60
    on_h = np.abs((seeds.imag + 1.0) / hy - np.round((seeds.imag + 1.0) / hy)) < 1e-9
    on_v = np.abs((seeds.real + 1.0) / hx - np.round((seeds.real + 1.0) / hx)) < 1e-9
    assert np.all(on_h | on_v)
    # order: horizontal edges first (row-major), then vertical edges
    nh = np.sum(inside[:, 1:] != inside[:, :-1])
    assert np.all(on_h[:nh]) and np.all(np.diff(np.round((seeds[:nh].imag + 1.0) / hy)) >= 0)
    # a grid point exactly on the level set (sigma == eps) is inside: the seed is that point
    g2 = W.Grid(-1.0, 1.0, 0.0, 0.0, 21, 1)
    s2 = np.abs(oracle.grid_points(g2))
    sd = oracle.contour_seeds(g2, s2, 0.5)
    np.testing.assert_allclose(np.sort(sd.real), [-0.5, 0.5], atol=1e-15)


def test_trace_contour_circles():
    # normal A: sigma_min(z) = dist(z, spectrum), so near an isolated eigenvalue a the
    # eps-level curve is the circle |z - a| = eps (Sec. 2, resolvent-norm definition)
    a = np.array([0.4 + 0.1j, -0.3 - 0.2j, 5.0])
    band = W.diagonal(a)
    eps, h = 1e-2, 1e-3
    pts, cnt, fl = oracle.trace_contour(band, [a[0] + 1.2e-2, a[1] - 0.9e-2j], eps, h, max_points=200)
    assert list(fl) == [oracle.TRACE_CLOSED, oracle.TRACE_CLOSED]
    for t in range(2):
        p = pts[t, :cnt[t]]
        assert np.all(np.abs(np.abs(p - a[t]) - eps) < 1e-10)
        # a tangent step of length h, then a radial correction: each step turns by
        # atan(h / eps), so consecutive points are 2 eps sin(atan(h / eps) / 2) apart and a full
        # turn takes 2 pi / atan(h / eps) steps
        th = np.arctan(h / eps)
        np.testing.assert_allclose(np.abs(np.diff(p)), 2 * eps * np.sin(th / 2), rtol=1e-6)
        assert abs(cnt[t] - 2 * np.pi / th) <= 2
        # counterclockwise around the region sigma < eps
        ang = np.unwrap(np.angle(p - a[t]))
        assert np.all(np.diff(ang) > 0)
    # the box stops a tracer at the first point outside it, which is stored
    pts, cnt, fl = oracle.trace_contour(band, [a[0] + 1.2e-2], eps, h, max_points=200,
                                        box=(a[0].real - 1.0, a[0].real + 1.0, a[0].imag - 1.0, a[0].imag + 0.005))
    assert fl[0] == oracle.TRACE_LEFT_BOX and pts[0, cnt[0] - 1].imag > a[0].imag + 0.005
    assert np.all(pts[0, :cnt[0] - 1].imag <= a[0].imag + 0.005)
    pts, cnt, fl = oracle.trace_contour(band, [a[0] + 1.2e-2], eps, h, max_points=10)
    assert fl[0] == oracle.TRACE_MAX_POINTS and cnt[0] == 10


def test_trace_contour_nonnormal_points_lie_on_the_curve():
    # Grcar n = 40: every traced point has sigma_min = eps by LAPACK's SVD (an opinion
    # independent of the Jacobi SVD the tracer uses), and consecutive points are about h apart
    band = W.grcar(40)
    A = W.to_dense(band)
    eps, h = 1e-2, 0.02
    pts, cnt, fl = oracle.trace_contour(band, [0.3 + 1.9j], eps, h, max_points=25)
    p = pts[0, :cnt[0]]
    assert cnt[0] == 25 and fl[0] == oracle.TRACE_MAX_POINTS
    s = np.array([np.linalg.svd(z * np.eye(40) - A, compute_uv=False)[-1] for z in p])
    assert np.all(np.abs(s / eps - 1) < 1e-6)
    d = np.abs(np.diff(p))
    assert np.all((d > 0.9 * h) & (d < 1.1 * h))


# ----------------------------------------------------------------------------- pair orders

@pytest.mark.parametrize("n", [7, 8, 13, 40, 41, 64])
def test_round_robin_order_small(n):
    """The round-robin (tournament) pair order reaches the same singular values as the cyclic
    order and as LAPACK, at even and odd n (odd n: one dummy player sits out each round)."""
    band = W.random_banded(n, 2, 3, seed=70 + n)
    z = np.array([0.3 - 0.2j, 1.7 + 0.9j])
    rr = oracle.sigma_min(band, z, all_sv=True, parallel_pairs=True, nthreads=4)
    cy = oracle.sigma_min(band, z, all_sv=True, parallel_pairs=False)
    A = W.to_dense(band)
    for k, zz in enumerate(z):
        ref = np.sort(np.linalg.svd(zz * np.eye(n) - A, compute_uv=False))
        t = _tol(band, ref[-1])
        assert np.max(np.abs(np.sort(rr["sall"][k]) - ref)) <= t
        assert np.max(np.abs(np.sort(rr["sall"][k]) - np.sort(cy["sall"][k]))) <= t
        assert abs(rr["sigma"][k] - ref[0]) <= _tol(band, ref[0])


@pytest.mark.parametrize("n", [512, 513])
def test_round_robin_order_large(n):
    """At n >= 512 (where the round-robin order is the default for few shifts) against LAPACK
    and, for a normal matrix, against the closed form dist(z, spectrum)."""
    band = W.random_banded(n, 1, 2, seed=n)
    z = np.array([0.4 + 0.1j])
    rr = oracle.sigma_min(band, z, all_sv=True, nthreads=8)        # default order at this size
    ref = np.sort(np.linalg.svd(z[0] * np.eye(n) - W.to_dense(band), compute_uv=False))
    assert np.max(np.abs(np.sort(rr["sall"][0]) - ref)) <= _tol(band, ref[-1])
    H = W.hermitian_toeplitz_tridiag(n, 0.1, 0.6 - 0.3j)
    lam = 0.1 + 2 * abs(0.6 - 0.3j) * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    zz = np.array([0.05 + 0.02j, 1.5 - 0.4j])
    s = oracle.sigma_min(H, zz, parallel_pairs=True, nthreads=8)["sigma"]
    assert np.allclose(s, np.min(np.abs(zz[:, None] - lam[None]), axis=1), atol=_tol(H), rtol=0)


# ----------------------------------------------------------------------------- planted mistakes

MUTANTS = {
    "conj_dropped": ("mp[i] = c * a - sec * b;", "mp[i] = c * a - se * b;"),
    "rotation_sign": ("mq[i] = se * a + c * b;", "mq[i] = se * a - c * b;"),
    "zeta_sign": ("double zeta = (beta - alpha) / (2.0 * g);", "double zeta = (alpha - beta) / (2.0 * g);"),
    "shift_sign": ("M[i + j * n] = -ab[ku + i - j + j * ldab];", "M[i + j * n] = ab[ku + i - j + j * ldab];"),
    "band_transposed": ("M[i + j * n] = -ab[ku + i - j + j * ldab];", "M[j + i * n] = -ab[ku + i - j + j * ldab];"),
    "shift_dropped": ("M[j + j * n] += z;", "M[j + j * n] += 0;"),
    "early_stop": ("double tau = (double)n * ldexp(1.0, -53);", "double tau = (double)n * ldexp(1.0, -12);"),
    "max_not_min": ("if (s < smin) {", "if (s > smin || smin == INFINITY) {"),
    "gamma_unconjugated": ("gamma += conj(mp[i]) * mq[i];", "gamma += mp[i] * mq[i];"),
    "u_unnormalised": ("u[r] = (smin > 0.0) ? M[r + imin * n] * ph / smin : 0.0;",
                       "u[r] = (smin > 0.0) ? M[r + imin * n] * ph : 0.0;"),
    # the round-robin pair order: a dropped slot, a wrong rotation modulus, a real player
    # treated as the dummy, a round missing
    "rr_slot0_dropped": ("for (int64_t k = 0; k < m / 2; ++k) {", "for (int64_t k = 1; k < m / 2; ++k) {"),
    "rr_mod_m": ("x = 1 + ((r + k) % (m - 1));", "x = 1 + ((r + k) % m);"),
    "rr_last_player_skipped": ("if (b >= n)", "if (b >= n - 1)"),
    "rr_round_missing": ("for (int64_t r = 0; r < m - 1; ++r) {", "for (int64_t r = 0; r < m - 2; ++r) {"),
}


def _pin_suite_passes(lib):
    """A compact version of the pins above, run against a given shared object."""
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.oracle_sigma_min.argtypes = [i64, i64, i64, P, i64, i64, P, P, P, P, P, P, ctypes.c_int, ctypes.c_int]

    def smin(band, z, vec=False, rr=0, sall=None):
        z = np.ascontiguousarray(np.asarray(z, dtype=complex))
        s = np.empty(z.size)
        u = np.empty((z.size, band.n), complex) if vec else None
        v = np.empty((z.size, band.n), complex) if vec else None
        sw = np.empty(z.size, np.int32)
        ab = np.ascontiguousarray(band.ab)
        p = lambda a: None if a is None else a.ctypes.data_as(P)
        st = lib.oracle_sigma_min(band.n, band.kl, band.ku, p(ab), band.kl + band.ku + 1, z.size, p(z), p(s),
                                  p(sall), p(u), p(v), p(sw), 2, rr)
        return st, s, u, v

    try:
        rng = _rng(99)
        vals = rng.standard_normal(9) + 1j * rng.standard_normal(9)
        z = rng.standard_normal(6) + 1j * rng.standard_normal(6)
        st, s, _, _ = smin(W.diagonal(vals), z)
        if st or not np.allclose(s, np.min(np.abs(z[:, None] - vals[None]), axis=1), atol=1e-12):
            return False
        n = 20
        H = W.hermitian_toeplitz_tridiag(n, 0.3, 0.7 + 0.2j)
        lam = 0.3 + 2 * abs(0.7 + 0.2j) * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
        st, s, _, _ = smin(H, z)
        if st or not np.allclose(s, np.min(np.abs(z[:, None] - lam[None]), axis=1), atol=1e-11):
            return False
        band = W.random_banded(9, 2, 1, seed=3)
        A = W.to_dense(band)
        st, s, u, v = smin(band, z, vec=True)
        if st:
            return False
        for k, zz in enumerate(z):
            M = zz * np.eye(9) - A
            if abs(s[k] - np.linalg.svd(M, compute_uv=False)[-1]) > 1e-11:
                return False
            if np.linalg.norm(M @ v[k] - s[k] * u[k]) > 1e-10 or abs(np.linalg.norm(u[k]) - 1) > 1e-10:
                return False
        # the round-robin order, even and odd n: every singular value against LAPACK
        for n in (10, 11):
            band = W.random_banded(n, 1, 2, seed=n)
            A = W.to_dense(band)
            sall = np.empty((z.size, n))
            st, s, _, _ = smin(band, z, rr=1, sall=sall)
            if st:
                return False
            for k, zz in enumerate(z):
                ref = np.sort(np.linalg.svd(zz * np.eye(n) - A, compute_uv=False))
                if np.max(np.abs(np.sort(sall[k]) - ref)) > 1e-11 or abs(s[k] - ref[0]) > 1e-11:
                    return False
        return True
    except Exception:
        return False


def test_oracle_mutants_are_caught():
    src = open(os.path.join(os.path.dirname(oracle.__file__), "jacobi.c")).read()
    tmp = tempfile.mkdtemp(prefix="oracle_mut_")
    try:
        # the unmodified source passes the compact suite
        libs = {}
        for name, (old, new) in [("original", ("", ""))] + list(MUTANTS.items()):
            if name != "original":
                assert src.count(old) >= 1, name
            text = src if name == "original" else src.replace(old, new, 1)
            c = os.path.join(tmp, name + ".c")
            so = os.path.join(tmp, name + ".so")
            open(c, "w").write(text)
            subprocess.check_call(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", c, "-o", so, "-lm"])
            libs[name] = ctypes.CDLL(so)
        assert _pin_suite_passes(libs.pop("original"))
        survivors = [name for name, lib in libs.items() if _pin_suite_passes(lib)]
        assert survivors == [], survivors
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
