"""Seeded synthetic workloads (inputs only).

Band storage used everywhere in this repository (LAPACK general-band, "GB"):
a C-contiguous ``numpy.complex128`` array ``ab`` of shape ``(n, kl + ku + 1)``
with ``ab[j, ku + i - j] = A[i, j]`` for ``max(0, j - ku) <= i <= min(n - 1, j + kl)``.
In memory this is exactly LAPACK's column-major ``AB(ldab = kl + ku + 1, n)``.
Entries of ``ab`` that fall outside the matrix are zero.

Matrix families follow the paper's setting (banded non-normal A, Sec. 1 and
the training generator of Sec. 3.3, eq. (matrix)) and the five measured
workloads; grids follow Sec. 2.1 (z_ij = x_j + i*y_i on [a,b] x [c,d]).
Random draws use ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

SEED_BASE = 2605_04550

__all__ = [
    "Band", "Grid", "SEED_BASE", "band_from_rows", "grcar", "toeplitz", "random_banded",
    "diagonal", "jordan", "jordan_perturbed", "hermitian_toeplitz_tridiag", "band_poly_hermitian",
    "circulant_full", "gershgorin_box", "paper_training_matrix", "annulus_list",
    "random_mask", "workload", "WORKLOADS", "batch_workload", "paper_label_workload", "to_dense",
]


@dataclasses.dataclass
class Band:
    """A banded n x n complex matrix in GB storage (see module docstring)."""
    ab: np.ndarray
    n: int
    kl: int
    ku: int
    real: bool = False          # all entries have zero imaginary part

    def __post_init__(self):
        self.ab = np.ascontiguousarray(self.ab, dtype=np.complex128)
        assert self.ab.shape == (self.n, self.kl + self.ku + 1), self.ab.shape

    @property
    def fro(self) -> float:
        return float(np.sqrt(np.sum(np.abs(self.ab) ** 2)))


@dataclasses.dataclass
class Grid:
    """Grid parameters of Sec. 2.1: x in [a, b] (nx points), y in [c, d] (ny points).

    Only parameters live here; each side (oracle, GPU library) forms the points
    itself.  Convention: inclusive end points, row index <-> y, column index <-> x,
    outputs row-major [ny][nx]; a single point along an axis sits at a (or c).
    """
    a: float
    b: float
    c: float
    d: float
    nx: int
    ny: int

    @property
    def npts(self) -> int:
        return self.nx * self.ny


def to_dense(band: Band) -> np.ndarray:
    """Dense copy of a band (input-format conversion for tests)."""
    n, kl, ku = band.n, band.kl, band.ku
    A = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            A[i, j] = band.ab[j, ku + i - j]
    return A


def band_from_rows(n: int, kl: int, ku: int, diags: Dict[int, object], real: bool = False) -> Band:
    """Build a band from diagonals: ``diags[d][i] = A[i, i + d]`` (d = j - i, scalar or array)."""
    ab = np.zeros((n, kl + ku + 1), dtype=np.complex128)
    for d, vals in diags.items():
        assert -kl <= d <= ku, d
        rows = np.arange(max(0, -d), min(n, n - d))
        v = np.broadcast_to(np.asarray(vals, dtype=np.complex128), (n,))
        for i in rows:
            j = i + d
            ab[j, ku + i - j] = v[i]
    return Band(ab, n, kl, ku, real)


def grcar(n: int, k: int = 3) -> Band:
    """Grcar matrix: -1 on the subdiagonal, +1 on the diagonal and k superdiagonals."""
    diags = {-1: -1.0}
    for d in range(0, k + 1):
        diags[d] = 1.0
    return band_from_rows(n, 1, k, diags, real=True)


def toeplitz(n: int, sub: complex, diag: complex, sup: complex) -> Band:
    """Tridiagonal Toeplitz matrix (sub, diag, super)."""
    real = all(complex(v).imag == 0 for v in (sub, diag, sup))
    return band_from_rows(n, 1, 1, {-1: sub, 0: diag, 1: sup}, real=real)


def diagonal(vals) -> Band:
    vals = np.asarray(vals, dtype=np.complex128)
    return band_from_rows(len(vals), 0, 0, {0: vals}, real=bool(np.all(vals.imag == 0)))


def _cn(rng, size) -> np.ndarray:
    """Complex normal CN(0,1): real and imaginary parts independent N(0, 1/2)."""
    return (rng.standard_normal(size) + 1j * rng.standard_normal(size)) * math.sqrt(0.5)


def random_banded(n: int, kl: int, ku: int, seed: int, scale: float = 1.0,
                  diag_uniform: float = 0.0) -> Band:
    """Entries on offsets -kl..ku i.i.d. CN(0,1)*scale; diagonal += U[-diag_uniform, diag_uniform]."""
    rng = np.random.default_rng(seed)
    ab = _cn(rng, (n, kl + ku + 1)) * scale
    if diag_uniform:
        ab[:, ku] += rng.uniform(-diag_uniform, diag_uniform, n)
    # zero the slots that fall outside the matrix (row i = r - ku + j)
    i = np.arange(kl + ku + 1)[None, :] - ku + np.arange(n)[:, None]
    ab[(i < 0) | (i >= n)] = 0
    return Band(ab, n, kl, ku, False)


def jordan(n: int = 32) -> Band:
    """Sec. 2 example: n x n Jordan block with ones on the subdiagonal (all eigenvalues 0)."""
    return band_from_rows(n, 1, 0, {-1: 1.0}, real=True)


def jordan_perturbed(n: int = 32, delta: float = 0.01) -> Band:
    """Sec. 2 example matrix B: the Jordan block plus ``delta`` in entry (1, n) (first row, last column)."""
    kl, ku = 1, n - 1
    b = band_from_rows(n, kl, ku, {-1: 1.0}, real=True)
    b.ab[n - 1, ku + 0 - (n - 1)] = delta
    return b


def hermitian_toeplitz_tridiag(n: int, a: float, b: complex) -> Band:
    """Hermitian tridiagonal Toeplitz H: diagonal a (real), superdiagonal b, subdiagonal conj(b)."""
    return band_from_rows(n, 1, 1, {-1: np.conj(b), 0: a, 1: b})


def band_poly_hermitian(n: int, a: float, b: complex, coeffs) -> Band:
    """p(H) for H = hermitian_toeplitz_tridiag(n, a, b) and complex polynomial coefficients
    ``coeffs`` (constant term first).  p(H) is normal with bandwidth deg p on each side.
    Built by dense products (input construction only)."""
    H = to_dense(hermitian_toeplitz_tridiag(n, a, b))
    P = np.zeros_like(H)
    Hk = np.eye(n, dtype=np.complex128)
    for c in coeffs:
        P = P + c * Hk
        Hk = Hk @ H
    deg = len(coeffs) - 1
    ab = np.zeros((n, 2 * deg + 1), dtype=np.complex128)
    for j in range(n):
        for i in range(max(0, j - deg), min(n, j + deg + 1)):
            ab[j, deg + i - j] = P[i, j]
    return Band(ab, n, deg, deg, False)


def circulant_full(col0) -> Band:
    """Circulant matrix C[i, j] = col0[(i - j) mod n], stored as a full band (kl = ku = n - 1)."""
    col0 = np.asarray(col0, dtype=np.complex128)
    n = len(col0)
    ab = np.zeros((n, 2 * n - 1), dtype=np.complex128)
    ku = n - 1
    for j in range(n):
        for i in range(n):
            ab[j, ku + i - j] = col0[(i - j) % n]
    return Band(ab, n, n - 1, n - 1, bool(np.all(col0.imag == 0)))


def gershgorin_box(band: Band):
    """Bounding box [a, b] x [c, d] of the row Gershgorin discs (centre a_ii, radius sum_{j != i} |a_ij|)."""
    n, kl, ku = band.n, band.kl, band.ku
    centre = band.ab[:, ku].copy()            # ab[j, ku] = A[j, j]
    radius = np.zeros(n)
    for r in range(kl + ku + 1):
        if r == ku:
            continue
        j = np.arange(n)
        i = r - ku + j                         # ab[j, r] = A[i, j]
        ok = (i >= 0) & (i < n)
        np.add.at(radius, i[ok], np.abs(band.ab[j[ok], r]))
    return (float(np.min(centre.real - radius)), float(np.max(centre.real + radius)),
            float(np.min(centre.imag - radius)), float(np.max(centre.imag + radius)))


def _grid_xy(grid: Grid):
    xs = np.array([grid.a + (grid.b - grid.a) * j / (grid.nx - 1) if grid.nx > 1 else grid.a
                   for j in range(grid.nx)])
    ys = np.array([grid.c + (grid.d - grid.c) * i / (grid.ny - 1) if grid.ny > 1 else grid.c
                   for i in range(grid.ny)])
    return xs, ys


def annulus_list(grid: Grid, seed: int, half_width: float = 1.0 / math.pi):
    """Restricted point set: grid points with ||z| - 1| <= half_width, as a uint8 mask [ny][nx]
    and as a seeded random permutation of their flat indices (the list form)."""
    xs, ys = _grid_xy(grid)
    X, Y = np.meshgrid(xs, ys)
    r = np.hypot(X, Y)
    mask = (np.abs(r - 1.0) <= half_width).astype(np.uint8)
    idx = np.flatnonzero(mask.ravel())
    rng = np.random.default_rng(seed)
    return mask, rng.permutation(idx).astype(np.int64)


def random_mask(grid: Grid, count: int, seed: int):
    """Exactly ``count`` grid points chosen without replacement (uint8 mask [ny][nx])."""
    rng = np.random.default_rng(seed)
    idx = rng.choice(grid.npts, size=count, replace=False)
    mask = np.zeros(grid.npts, dtype=np.uint8)
    mask[idx] = 1
    return mask.reshape(grid.ny, grid.nx)


def paper_training_matrix(seed: int, n: int = 64, max_tries: int = 1000) -> Band:
    """Sec. 3.3, eq. (matrix): bandwidth beta ~ U{1..4}; A_ij ~ U{-1, 0, 1} for |i-j| <= beta, else 0;
    rejected if A equals its transpose or if cond(A) >= 1e8."""
    rng = np.random.default_rng(seed)
    for _ in range(max_tries):
        beta = int(rng.integers(1, 5))
        A = np.zeros((n, n))
        for i in range(n):
            for j in range(max(0, i - beta), min(n, i + beta + 1)):
                A[i, j] = rng.integers(-1, 2)
        if np.array_equal(A, A.T):
            continue
        s = np.linalg.svd(A, compute_uv=False)
        if s[-1] == 0 or s[0] / s[-1] >= 1e8:
            continue
        ab = np.zeros((n, 2 * beta + 1), dtype=np.complex128)
        for j in range(n):
            for i in range(max(0, j - beta), min(n, j + beta + 1)):
                ab[j, beta + i - j] = A[i, j]
        return Band(ab, n, beta, beta, True)
    raise RuntimeError("no admissible matrix")


# --------------------------------------------------------------------------------------
# The measured workloads.  Each returns a dict with the band, the grid and (where the
# workload has one) the restricted point set.

def _w_grcar100():
    return dict(name="grcar100", band=grcar(100), grid=Grid(-1.5, 3.0, -3.5, 3.5, 64, 64))


def _w_toeplitz2000():
    grid = Grid(-2.0, 2.0, -2.0, 2.0, 256, 256)
    mask, lst = annulus_list(grid, SEED_BASE + 2)
    return dict(name="toeplitz2000", band=toeplitz(2000, 0.25, 0.0, 1.0), grid=grid,
                mask=mask, list=lst)


def _w_random10k():
    band = random_banded(10000, 2, 3, SEED_BASE + 3, scale=1.0 / math.sqrt(6.0), diag_uniform=1.0)
    a, b, c, d = gershgorin_box(band)
    return dict(name="random10k", band=band, grid=Grid(a, b, c, d, 512, 512))


def batch_workload(nmat: int = 64, grid_n: int = 128, frac: float = 0.3, nmin: int = 500,
                   nmax: int = 20000):
    """Batch of banded matrices of uneven size and bandwidth, each with its own grid on its
    Gershgorin box and a random mask of round(frac * grid_n^2) points."""
    rng = np.random.default_rng(SEED_BASE + 4)
    mats = []
    count = int(round(frac * grid_n * grid_n))
    for m in range(nmat):
        n = int(rng.integers(nmin, nmax + 1))
        kl = int(rng.integers(1, 5))
        ku = int(rng.integers(1, 5))
        band = random_banded(n, kl, ku, SEED_BASE + 1000 + m)
        a, b, c, d = gershgorin_box(band)
        grid = Grid(a, b, c, d, grid_n, grid_n)
        mats.append(dict(band=band, grid=grid, mask=random_mask(grid, count, SEED_BASE + 2000 + m)))
    return dict(name="batch64", mats=mats)


def _w_grcar4000():
    rng = np.random.default_rng(SEED_BASE + 5)
    grid = Grid(-1.5, 3.0, -3.5, 3.5, 256, 256)
    return dict(name="grcar4000", band=grcar(4000), grid=grid,
                weights=rng.standard_normal(grid.npts), eps=1e-3)


def paper_label_workload(nmat: int = 500, first: int = 0):
    """The label-generation setting of Sec. 3.3: matrices of the class of eq. (matrix), n = 64,
    each labelled on a 100 x 100 grid over [-4, 4] x [-4, 4] with eps = 0.01 (z sensitive iff
    sigma_min(zI - A) <= eps).  Matrix m uses seed base + 6000 + m."""
    grid = Grid(-4.0, 4.0, -4.0, 4.0, 100, 100)
    mats = [paper_training_matrix(SEED_BASE + 6000 + m) for m in range(first, first + nmat)]
    return dict(name="paper_labels", mats=mats, grid=grid, eps=0.01)


WORKLOADS = {
    "grcar100": _w_grcar100,
    "toeplitz2000": _w_toeplitz2000,
    "random10k": _w_random10k,
    "batch64": batch_workload,
    "grcar4000": _w_grcar4000,
}


def workload(name: str):
    return WORKLOADS[name]()
