"""CPU oracle for the sigma_min(zI - A) hot path.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and by
the benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU library (its own C source, its own grid and band handling); the two
meet only through the seeded inputs of the ``workloads`` package.

Contents (each function names the passage of the paper it follows):
  * ``sigma_min``      -- dense one-sided Jacobi SVD per shift (``jacobi.c``), Sec. 2.1 and
                          the third form of the pseudospectrum definition (Sec. 2).
  * ``smallest_pair_lapack`` -- the same sigma_min with its singular pair from LAPACK's dense
                          SVD (numpy), for the n = 4000 gradient values; checked against
                          ``sigma_min`` at small n.
  * ``grid_points``    -- the shift grid G of Sec. 2.1.
  * ``compact_mask``   -- the restricted set R of Sec. 4 as an index list.
  * ``sensitive``      -- the sensitive zone S_eps, Sec. 2.1 eq. (sensitive_zone).
  * ``adjoint``        -- gradients of sigma_min from the singular pair (first-order
                          perturbation of a simple singular value; the paper is silent).
  * ``newton_step``    -- one Newton step on ln(sigma/eps) toward the eps-level curve
                          (the level curve of Sec. 2.1; the paper is silent on refinement).
  * ``contour_seeds``  -- starting points on the eps-level curve from sign changes of
                          sigma - eps along grid edges (Sec. 2.1 level curve).
  * ``count_below``    -- number of singular values of zI - A below t, by the inertia of a
                          banded Hermitian augmented matrix (``inertia.c``); certifies
                          sigma_min at sizes where a dense SVD per shift is too slow.
  * ``trace_contour``  -- points along the eps-level curve from seeds: a step along the
                          tangent, then Newton steps back onto the curve (Sec. 2.1 level
                          curve; the paper does not say how to follow it).
  * ``mask``           -- submodule: the classifier of Sec. 3.2 and its hierarchical use over a
                          grid (Sec. 3.5), the producer of the restricted set R (Sec. 4).
Pins: every function here is checked in ``tests/test_oracle_pins.py`` against
closed forms, invariants, brute force and the paper's Jordan example; the ``mask``
submodule in ``tests/test_oracle_mask_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "jacobi.c"), os.path.join(_HERE, "inertia.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP, no LAPACK)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", *_SRCS,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_sigma_min.argtypes = [i64, i64, i64, P, i64, i64, P, P, P, P, P, P,
                                         ctypes.c_int, ctypes.c_int]
        lib.oracle_sigma_min.restype = ctypes.c_int
        lib.oracle_svd_dense.argtypes = [i64, P, P, P, P, P]
        lib.oracle_svd_dense.restype = ctypes.c_int
        lib.oracle_count_below.argtypes = [i64, i64, i64, P, i64, i64, P, P, P, ctypes.c_int]
        lib.oracle_count_below.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def sigma_min(band, z, want_vectors: bool = False, all_sv: bool = False, nthreads: int | None = None,
              parallel_pairs: bool | None = None):
    """sigma_min(zI - A) at each shift in ``z`` (Sec. 2.1: sigma_min(z) = s_n of the SVD).

    ``band`` has attributes ab (GB, shape (n, kl+ku+1)), n, kl, ku.  Returns a dict with
    ``sigma`` [npts]; ``sall`` [npts, n] (unsorted) if ``all_sv``; ``u``, ``v`` [npts, n]
    (phase: first max-modulus entry of v real positive) if ``want_vectors``; ``sweeps``.
    """
    lib = _load()
    z = np.ascontiguousarray(np.atleast_1d(np.asarray(z, dtype=np.complex128)))
    ab = np.ascontiguousarray(band.ab, dtype=np.complex128)
    n, kl, ku = int(band.n), int(band.kl), int(band.ku)
    npts = z.size
    nthreads = nthreads or default_threads()
    if parallel_pairs is None:
        parallel_pairs = n >= 512 and npts < nthreads
    sigma = np.empty(npts)
    sall = np.empty((npts, n)) if all_sv else None
    u = np.empty((npts, n), dtype=np.complex128) if want_vectors else None
    v = np.empty((npts, n), dtype=np.complex128) if want_vectors else None
    sweeps = np.empty(npts, dtype=np.int32)
    st = lib.oracle_sigma_min(n, kl, ku, _ptr(ab), kl + ku + 1, npts, _ptr(z), _ptr(sigma), _ptr(sall),
                              _ptr(u), _ptr(v), _ptr(sweeps), int(nthreads), int(bool(parallel_pairs)))
    if st != 0:
        raise RuntimeError("oracle Jacobi failed (status %d)" % st)
    out = dict(sigma=sigma, sweeps=sweeps)
    if all_sv:
        out["sall"] = sall
    if want_vectors:
        out["u"], out["v"] = u, v
    return out


def svd_dense(M):
    """All singular values (unsorted, column order) and U, V of a dense complex matrix."""
    lib = _load()
    M = np.asarray(M, dtype=np.complex128)
    n = M.shape[0]
    Mf = np.asfortranarray(M)
    s = np.empty(n)
    U = np.empty((n, n), dtype=np.complex128, order="F")
    V = np.empty((n, n), dtype=np.complex128, order="F")
    sw = np.empty(1, dtype=np.int32)
    st = lib.oracle_svd_dense(n, _ptr(Mf), _ptr(s), _ptr(U), _ptr(V), _ptr(sw))
    if st != 0:
        raise RuntimeError("oracle Jacobi failed (status %d)" % st)
    return s, U, V


def smallest_pair_lapack(band, z):
    """sigma_n, sigma_{n-1} and the singular pair (u, v) of sigma_n for each shift, from LAPACK's
    dense SVD of zI - A (Sec. 2.1: sigma_min(z) is the smallest singular value, with M v = sigma u).

    A second dense SVD beside the Jacobi one of ``sigma_min``, for sizes (n in the thousands)
    where the Jacobi sweeps take too long; the two are checked against each other at small n.
    Returns a dict with ``sigma``, ``s2`` [npts] and ``u``, ``v`` [npts, n]."""
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    n, kl, ku = int(band.n), int(band.kl), int(band.ku)
    A = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):                           # GB layout: ab[j, ku + i - j] = A[i, j]
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            A[i, j] = band.ab[j, ku + i - j]
    sig = np.empty(z.size)
    s2 = np.empty(z.size)
    u = np.empty((z.size, n), dtype=np.complex128)
    v = np.empty((z.size, n), dtype=np.complex128)
    for p, zz in enumerate(z):
        U, S, Vh = np.linalg.svd(zz * np.eye(n) - A)      # S descending
        sig[p] = S[-1]
        s2[p] = S[-2] if n > 1 else np.inf
        u[p] = U[:, -1]
        v[p] = np.conj(Vh[-1])
    return dict(sigma=sig, s2=s2, u=u, v=v)


def grid_points(grid) -> np.ndarray:
    """Sec. 2.1: z_ij = x_j + i*y_i, x_j in [a, b] (N_x points), y_i in [c, d] (N_y points).

    Inclusive end points (x_j = a + (b - a) j/(N_x - 1); a single point sits at a);
    flattened row-major, row index <-> y.
    """
    xs = np.array([grid.a + (grid.b - grid.a) * j / (grid.nx - 1) if grid.nx > 1 else grid.a
                   for j in range(grid.nx)], dtype=np.float64)
    ys = np.array([grid.c + (grid.d - grid.c) * i / (grid.ny - 1) if grid.ny > 1 else grid.c
                   for i in range(grid.ny)], dtype=np.float64)
    return (xs[None, :] + 1j * ys[:, None]).ravel()


def compact_mask(mask) -> np.ndarray:
    """Sec. 4: the restricted set R as the ascending flat indices of the nonzero mask entries."""
    return np.flatnonzero(np.asarray(mask).ravel()).astype(np.int64)


def sensitive(sigma, eps) -> np.ndarray:
    """Sec. 2.1 eq. (sensitive_zone): z is sensitive iff sigma_min(z) <= eps (inclusive)."""
    return (np.asarray(sigma) <= eps).astype(np.uint8)


def adjoint(band, u, v, grad_sigma):
    """Gradients of L = sum_p g_p sigma_p for sigma_p = sigma_min(z_p I - A), from the singular pairs.

    For a simple singular value, d sigma = Re(u^H dM v) with dM = dz I - dA.  In the
    conjugate-Wirtinger convention (d/dRe + i d/dIm):
        grad_z[p]   = g_p * conj(u_p^H v_p)
        grad_A[i,j] = -sum_p g_p * u_p[i] * conj(v_p[j])   (only on the band)
    Returns grad_z [npts] and grad_band in GB layout (shape of band.ab).
    """
    u = np.asarray(u, dtype=np.complex128)
    v = np.asarray(v, dtype=np.complex128)
    g = np.asarray(grad_sigma, dtype=np.float64)
    c = np.sum(np.conj(u) * v, axis=1)
    grad_z = g * np.conj(c)
    n, kl, ku = band.n, band.kl, band.ku
    gb = np.zeros_like(band.ab)
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            gb[j, ku + i - j] = -np.sum(g * u[:, i] * np.conj(v[:, j]))
    return grad_z, gb


def newton_step(z, sigma, grad_z, eps):
    """One Newton step on phi(z) = ln(sigma_min(z)/eps) along its gradient:
    z <- z - phi * (grad sigma / sigma) / |grad sigma / sigma|^2 = z - sigma ln(sigma/eps) g/|g|^2,
    with g = grad_z (conjugate-Wirtinger gradient of sigma_min)."""
    z = np.asarray(z, dtype=np.complex128)
    sigma = np.asarray(sigma, dtype=np.float64)
    g = np.asarray(grad_z, dtype=np.complex128)
    return z - sigma * np.log(sigma / eps) * g / np.abs(g) ** 2


def count_below(band, z, t, nthreads: int | None = None) -> np.ndarray:
    """#{singular values of z_p I - A below t_p} for each point (inertia of
    [[-t I, M], [M^H, -t I]] by a banded L D L^H, ``inertia.c``); -1 marks an exactly zero pivot."""
    lib = _load()
    z = np.ascontiguousarray(np.atleast_1d(z), dtype=np.complex128)
    t = np.ascontiguousarray(np.broadcast_to(np.asarray(t, dtype=np.float64), z.shape))
    ab = np.ascontiguousarray(band.ab, dtype=np.complex128)
    out = np.zeros(z.shape, dtype=np.int64)
    lib.oracle_count_below(band.n, band.kl, band.ku, _ptr(ab), band.kl + band.ku + 1, len(z), _ptr(z), _ptr(t),
                           _ptr(out), nthreads or default_threads())
    return out


def contour_seeds(grid, sigma, eps) -> np.ndarray:
    """Points on the eps-level curve of sigma_min (the curve the paper draws at log10 eps,
    Sec. 2.1), one per grid edge whose two end points lie on different sides of the
    inclusive test sigma <= eps.  On such an edge z1 -> z2 the seed is z1 + tau (z2 - z1),
    tau = (ln eps - ln s1) / (ln s2 - ln s1), linear interpolation of ln sigma (sigma is
    clamped to 2^-1022 before the logarithm).  Order: the horizontal edges (i, j)-(i, j+1)
    in row-major order of (i, j), then the vertical edges (i, j)-(i+1, j) likewise."""
    nx, ny = int(grid.nx), int(grid.ny)
    s = np.asarray(sigma, dtype=np.float64).reshape(ny, nx)
    z = grid_points(grid).reshape(ny, nx)
    inside = s <= eps
    ls = np.log(np.maximum(s, 2.0 ** -1022))
    le = np.log(eps)
    out = []
    for (a, b) in (((slice(None), slice(0, nx - 1)), (slice(None), slice(1, nx))),
                   ((slice(0, ny - 1), slice(None)), (slice(1, ny), slice(None)))):
        sel = inside[a] != inside[b]
        l1, l2 = ls[a][sel], ls[b][sel]
        z1, z2 = z[a][sel], z[b][sel]
        tau = (le - l1) / (l2 - l1)
        out.append(z1 + tau * (z2 - z1))
    return np.concatenate(out)



TRACE_CLOSED, TRACE_LEFT_BOX, TRACE_NEWTON_FAILED, TRACE_MAX_POINTS = 1, 2, 4, 8


def trace_contour(band, seeds, eps, h, max_points, newton_steps=2, box=None):
    """Follow the eps-level curve sigma_min(zI - A) = eps (the boundary of the
    eps-pseudospectrum that Sec. 2.1 draws as the level curve log10 eps) from each seed.

    With g = grad sigma_min (conjugate-Wirtinger, from the singular pair, ``adjoint``) the
    curve's tangent is i g / |g|.  A tracer first takes 2 newton_steps + 2 Newton steps
    (``newton_step``) from its seed onto the curve (a seed may lie a grid spacing away): that
    is point 0.  Point k then comes from
    point k-1 by a step of length h along the tangent (computed at point k-1) followed by
    ``newton_steps`` Newton steps; at every point sigma and g are evaluated once more.  A
    tracer stops, with the flag set, when a corrected point misses the curve
    (|ln(sigma/eps)| > 1e-6: TRACE_NEWTON_FAILED, the point is not stored), when a point lies
    outside the box (a, b, c, d) (TRACE_LEFT_BOX, stored), when point k >= 3 lies within h of
    point 0 (TRACE_CLOSED, stored), or after max_points points (TRACE_MAX_POINTS).
    Returns points [nseed, max_points] (unused entries 0), count [nseed], flags [nseed]."""
    seeds = np.atleast_1d(np.asarray(seeds, dtype=np.complex128))
    m = len(seeds)

    def evaluate(z):
        r = sigma_min(band, z, want_vectors=True)
        g, _ = adjoint(band, r["u"], r["v"], np.ones(len(z)))
        return r["sigma"], g

    def correct(z, steps):
        for _ in range(steps):
            s, g = evaluate(z)
            z = newton_step(z, s, g, eps)
        s, g = evaluate(z)
        return z, s, g

    pts = np.zeros((m, max_points), dtype=np.complex128)
    count = np.zeros(m, dtype=np.int32)
    flags = np.zeros(m, dtype=np.int32)
    for t in range(m):
        z = np.array([seeds[t]])
        z0 = None
        g = None
        for k in range(max_points):
            if k > 0:
                z = z + h * 1j * g / np.abs(g)
            z, s, g = correct(z, newton_steps if k > 0 else 2 * newton_steps + 2)
            if not (np.isfinite(s[0]) and s[0] > 0 and abs(np.log(s[0] / eps)) <= 1e-6):
                flags[t] |= TRACE_NEWTON_FAILED
                break
            pts[t, k] = z[0]
            count[t] = k + 1
            if k == 0:
                z0 = z[0]
            if box is not None:
                a, b, c, d = box
                if not (a <= z[0].real <= b and c <= z[0].imag <= d):
                    flags[t] |= TRACE_LEFT_BOX
                    break
            if k >= 3 and abs(z[0] - z0) < h:
                flags[t] |= TRACE_CLOSED
                break
            if k == max_points - 1:
                flags[t] |= TRACE_MAX_POINTS
    return pts, count, flags
