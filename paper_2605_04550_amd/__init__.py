"""Python binding of the MI355X sigma_min(zI - A) library (``libps.so``, C ABI in include/ps.h).

The functions named ``ps_*`` mirror the C entry points one to one (argument
marshalling only); every step of the computation runs in the HIP kernels.  PyTorch
supplies device memory and the current stream.  Higher-level helpers
(``BandedMatrix``, ``sigma_min``, ``eval_grid``, ``SigmaMin``, ``newton_contour``)
live in ``paper_2605_04550_amd.api``.

There is no CPU fallback: if ``libps.so`` is missing this module raises on import of
any entry point.  Build it with ``python -m paper_2605_04550_amd.build``.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libps.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "ps.h")

PS_OK, PS_ERR_INVALID, PS_ERR_NONFINITE, PS_ERR_WORKSPACE, PS_ERR_HIP, PS_ERR_UNSUPPORTED = range(6)
PS_PT_CONVERGED, PS_PT_SINGULAR, PS_PT_MAXITER, PS_PT_UNDERFLOW, PS_PT_BISECT = 0, 1, 2, 4, 8
PS_TRACE_CLOSED, PS_TRACE_LEFT_BOX, PS_TRACE_NEWTON_FAILED, PS_TRACE_MAX_POINTS = 1, 2, 4, 8
PS_DEVICE_PTR, PS_REAL_A = 1, 2

STATUS_NAMES = {0: "PS_OK", 1: "PS_ERR_INVALID", 2: "PS_ERR_NONFINITE", 3: "PS_ERR_WORKSPACE", 4: "PS_ERR_HIP",
                5: "PS_ERR_UNSUPPORTED"}


class ps_c128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class ps_grid(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("b", ctypes.c_double), ("c", ctypes.c_double), ("d", ctypes.c_double),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64)]


class ps_opts(ctypes.Structure):
    _fields_ = [("tol_norm", ctypes.c_double), ("tol_rel", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("want_vectors", ctypes.c_int32), ("slots", ctypes.c_int32), ("check_shift", ctypes.c_int32),
                ("bisect", ctypes.c_int32), ("lanes", ctypes.c_int32), ("tests", ctypes.c_int32)]


class ps_mask_opts(ctypes.Structure):
    _fields_ = [("stride", ctypes.c_int32), ("dilate", ctypes.c_int32), ("coarse_q", ctypes.c_double),
                ("tau", ctypes.c_double)]


PS_MLP_NPARAM, PS_MLP_NGLOBAL = 59841, 30


class PsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32

_SIGNATURES = {
    "ps_opts_default": (None, [ctypes.POINTER(ps_opts)]),
    "ps_last_error": (ctypes.c_char_p, []),
    "ps_version": (ctypes.c_char_p, []),
    "ps_set_timing_events": (ctypes.c_int, [_P, _P]),
    "ps_create_banded": (ctypes.c_int, [_P, _I64, _I64, _I32, _I32, ctypes.c_uint32, _P, ctypes.POINTER(_P)]),
    "ps_destroy": (ctypes.c_int, [_P]),
    "ps_matrix_info": (ctypes.c_int, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                      ctypes.POINTER(ctypes.c_double)]),
    "ps_workspace_size": (ctypes.c_int, [_P, _I64, ctypes.POINTER(ps_opts), ctypes.POINTER(ctypes.c_size_t)]),
    "ps_eval_points": (ctypes.c_int, [_P, _P, _I64, ctypes.POINTER(ps_opts), _P, ctypes.c_size_t, _P, _P, _P, _P,
                                      _P, _P]),
    "ps_eval_points_noalloc": (ctypes.c_int, [_P, _P, _I64, ctypes.POINTER(ps_opts), _P, _P, _P, _P]),
    "ps_eval_grid": (ctypes.c_int, [_P, ctypes.POINTER(ps_grid), _P, ctypes.POINTER(ps_opts), _P, ctypes.c_size_t,
                                    _P, _P, _P, _P, _P, _P, _P, ctypes.c_double, _P, _P]),
    "ps_backward_workspace_size": (ctypes.c_int, [_P, _I64, ctypes.POINTER(ctypes.c_size_t)]),
    "ps_backward": (ctypes.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "ps_newton_workspace_size": (ctypes.c_int, [_P, _I64, ctypes.POINTER(ps_opts), ctypes.POINTER(ctypes.c_size_t)]),
    "ps_newton_contour": (ctypes.c_int, [_P, _P, _I64, ctypes.c_double, _I32, ctypes.POINTER(ps_opts), _P,
                                         ctypes.c_size_t, _P, _P, _P]),
    "ps_trace_workspace_size": (ctypes.c_int, [_P, _I64, ctypes.POINTER(ps_opts), ctypes.POINTER(ctypes.c_size_t)]),
    "ps_trace_contour": (ctypes.c_int, [_P, _P, _I64, ctypes.c_double, ctypes.c_double, _I32, _I32,
                                        ctypes.POINTER(ps_grid), ctypes.POINTER(ps_opts), _P, ctypes.c_size_t, _P, _P,
                                        _P, _P]),
    "ps_label_batch_workspace_size": (ctypes.c_int, [_P, ctypes.POINTER(ps_opts), ctypes.POINTER(ctypes.c_size_t)]),
    "ps_label_batch": (ctypes.c_int, [_P, ctypes.c_double, ctypes.POINTER(ps_opts), _P, ctypes.c_size_t, _P, _P, _P,
                                      _P]),
    "ps_label_workspace_size": (ctypes.c_int, [_P, ctypes.POINTER(ps_grid), ctypes.POINTER(ps_opts),
                                               ctypes.POINTER(ctypes.c_size_t)]),
    "ps_label_grid": (ctypes.c_int, [_P, ctypes.POINTER(ps_grid), ctypes.c_double, ctypes.POINTER(ps_opts), _P,
                                     ctypes.c_size_t, _P, _P, _P, _P]),
    "ps_contour_seeds_workspace_size": (ctypes.c_int, [ctypes.POINTER(ps_grid), ctypes.POINTER(ctypes.c_size_t)]),
    "ps_contour_seeds": (ctypes.c_int, [ctypes.POINTER(ps_grid), _P, ctypes.c_double, _P, _I64, _P, _P,
                                        ctypes.c_size_t, _P]),
    "ps_autotune": (ctypes.c_int, [_P, _P, _I64, ctypes.POINTER(ps_opts), _P]),
    "ps_autotune_batch": (ctypes.c_int, [_P, _P, ctypes.POINTER(ps_opts), _P]),
    "ps_plan_cache_clear": (None, []),
    "ps_create_batch": (ctypes.c_int, [_I32, ctypes.POINTER(_P), ctypes.POINTER(ps_grid), ctypes.POINTER(_P)]),
    "ps_destroy_batch": (ctypes.c_int, [_P]),
    "ps_batch_info": (ctypes.c_int, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "ps_batch_workspace_size": (ctypes.c_int, [_P, ctypes.POINTER(ps_opts), ctypes.POINTER(ctypes.c_size_t)]),
    "ps_eval_batch": (ctypes.c_int, [_P, _P, ctypes.POINTER(ps_opts), _P, ctypes.c_size_t, _P, _P, _P, _P, _P, _P]),
    "ps_mask_opts_default": (None, [ctypes.POINTER(ps_mask_opts)]),
    "ps_mlp_create": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.POINTER(_P), _P]),
    "ps_mlp_destroy": (ctypes.c_int, [_P]),
    "ps_mask_workspace_size": (ctypes.c_int, [ctypes.POINTER(ps_grid), ctypes.POINTER(ps_mask_opts),
                                              ctypes.POINTER(ctypes.c_size_t)]),
    "ps_mlp_prob": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), _P, _I64, _P, _I64, _P, ctypes.c_size_t, _P,
                                   _P]),
    "ps_mask_predict": (ctypes.c_int, [_P, ctypes.POINTER(ps_grid), ctypes.POINTER(ctypes.c_double), _P, _I64,
                                       ctypes.POINTER(ps_mask_opts), _P, ctypes.c_size_t, _P, _P, _P, _P, _P, _P]),
    "ps_mask_calibrate_workspace_size": (ctypes.c_int, [_I32, _I32, ctypes.POINTER(ctypes.c_size_t)]),
    "ps_mask_calibrate": (ctypes.c_int, [_I32, ctypes.POINTER(ps_grid), _P, _P, ctypes.POINTER(ctypes.c_double), _I32,
                                         _I32, _I32, ctypes.c_double, ctypes.c_double, _P, ctypes.c_size_t, _P, _P, _P,
                                         _P, _P]),
    "ps_mask_batch_workspace_size": (ctypes.c_int, [_I32, ctypes.POINTER(ps_grid), ctypes.POINTER(ps_mask_opts),
                                                    ctypes.POINTER(ctypes.c_size_t)]),
    "ps_mask_predict_batch": (ctypes.c_int, [_P, _I32, ctypes.POINTER(ps_grid), ctypes.POINTER(ctypes.c_double), _P,
                                             ctypes.POINTER(_I64), ctypes.POINTER(ps_mask_opts), _P, ctypes.c_size_t,
                                             _P, _P, _P, _P, _P, _P]),
}


def lib():
    """The loaded ``libps.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libps.so not found at %s; build it with `python -m paper_2605_04550_amd.build` "
                              "(there is no CPU fallback)" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != PS_OK:
        raise PsError(status, lib().ps_last_error().decode(errors="replace"))
    return status


def ps_last_error() -> str:
    return lib().ps_last_error().decode(errors="replace")


def ps_eval_points_noalloc(handle: int, z_ptr: int, npts: int, opts, sigma_ptr: int, info_ptr: int = 0,
                           iters_ptr: int = 0, stream: int = 0) -> None:
    """ps_eval_points with the library's fixed device scratch instead of a workspace (sigma only)."""
    _check(lib().ps_eval_points_noalloc(_P(handle), _P(z_ptr), npts, ctypes.byref(opts) if opts is not None else None,
                                        _P(sigma_ptr), _P(info_ptr or None), _P(iters_ptr or None), _P(stream)))


def ps_set_timing_events(start: int, end: int) -> None:
    """Measurement hook: hipEvent_t handles (ints, 0 = off) recorded around the bisection launches."""
    _check(lib().ps_set_timing_events(_P(start or None), _P(end or None)))


def ps_version() -> str:
    return lib().ps_version().decode()


def ps_opts_default(**overrides) -> ps_opts:
    o = ps_opts()
    lib().ps_opts_default(ctypes.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def ps_create_banded(ab_ptr: int, ldab: int, n: int, kl: int, ku: int, flags: int = 0, stream: int = 0) -> int:
    """Returns the opaque handle (an int).  ab_ptr: address of the GB band (host unless PS_DEVICE_PTR)."""
    h = _P()
    _check(lib().ps_create_banded(_P(ab_ptr), ldab, n, kl, ku, flags, _P(stream), ctypes.byref(h)))
    return h.value


def ps_destroy(handle: int) -> None:
    _check(lib().ps_destroy(_P(handle)))


def ps_matrix_info(handle: int):
    n, kl, ku, fro = _I64(), _I32(), _I32(), ctypes.c_double()
    _check(lib().ps_matrix_info(_P(handle), ctypes.byref(n), ctypes.byref(kl), ctypes.byref(ku), ctypes.byref(fro)))
    return n.value, kl.value, ku.value, fro.value


def ps_workspace_size(handle: int, npts: int, opts: ps_opts | None = None) -> int:
    b = ctypes.c_size_t()
    _check(lib().ps_workspace_size(_P(handle), npts, ctypes.byref(opts) if opts is not None else None,
                                   ctypes.byref(b)))
    return b.value


def ps_eval_points(handle, z_ptr, npts, opts, ws_ptr, ws_bytes, sigma_ptr, u_ptr=0, v_ptr=0, info_ptr=0,
                   iters_ptr=0, stream=0) -> None:
    _check(lib().ps_eval_points(_P(handle), _P(z_ptr), npts, ctypes.byref(opts) if opts is not None else None,
                                _P(ws_ptr), ws_bytes, _P(sigma_ptr), _P(u_ptr), _P(v_ptr), _P(info_ptr),
                                _P(iters_ptr), _P(stream)))


def ps_eval_grid(handle, grid: ps_grid, mask_ptr, opts, ws_ptr, ws_bytes, idx_ptr, count_ptr, sigma_ptr, u_ptr=0,
                 v_ptr=0, info_ptr=0, iters_ptr=0, eps=0.0, sens_ptr=0, stream=0) -> None:
    _check(lib().ps_eval_grid(_P(handle), ctypes.byref(grid), _P(mask_ptr),
                              ctypes.byref(opts) if opts is not None else None, _P(ws_ptr), ws_bytes, _P(idx_ptr),
                              _P(count_ptr), _P(sigma_ptr), _P(u_ptr), _P(v_ptr), _P(info_ptr), _P(iters_ptr),
                              float(eps), _P(sens_ptr), _P(stream)))


def ps_backward_workspace_size(handle: int, npts: int) -> int:
    b = ctypes.c_size_t()
    _check(lib().ps_backward_workspace_size(_P(handle), npts, ctypes.byref(b)))
    return b.value


def ps_backward(handle, npts, grad_sigma_ptr, u_ptr, v_ptr, grad_z_ptr, grad_band_ptr, ws_ptr, ws_bytes,
                stream=0) -> None:
    _check(lib().ps_backward(_P(handle), npts, _P(grad_sigma_ptr), _P(u_ptr), _P(v_ptr), _P(grad_z_ptr),
                             _P(grad_band_ptr), _P(ws_ptr), ws_bytes, _P(stream)))


def ps_newton_workspace_size(handle: int, npts: int, opts: ps_opts | None = None) -> int:
    b = ctypes.c_size_t()
    _check(lib().ps_newton_workspace_size(_P(handle), npts, ctypes.byref(opts) if opts is not None else None,
                                          ctypes.byref(b)))
    return b.value


def ps_newton_contour(handle, z_ptr, npts, eps, steps, opts, ws_ptr, ws_bytes, sigma_ptr, info_ptr=0,
                      stream=0) -> None:
    _check(lib().ps_newton_contour(_P(handle), _P(z_ptr), npts, float(eps), int(steps),
                                   ctypes.byref(opts) if opts is not None else None, _P(ws_ptr), ws_bytes,
                                   _P(sigma_ptr), _P(info_ptr), _P(stream)))


def ps_trace_workspace_size(handle: int, nseed: int, opts: ps_opts | None = None) -> int:
    b = ctypes.c_size_t()
    _check(lib().ps_trace_workspace_size(_P(handle), nseed, ctypes.byref(opts) if opts is not None else None,
                                         ctypes.byref(b)))
    return b.value


def ps_trace_contour(handle, seeds_ptr, nseed, eps, h, max_points, newton_steps, box, opts, ws_ptr, ws_bytes,
                     points_ptr, count_ptr, flags_ptr, stream=0) -> None:
    _check(lib().ps_trace_contour(_P(handle), _P(seeds_ptr), nseed, float(eps), float(h), int(max_points),
                                  int(newton_steps), ctypes.byref(box) if box is not None else None,
                                  ctypes.byref(opts) if opts is not None else None, _P(ws_ptr), ws_bytes,
                                  _P(points_ptr), _P(count_ptr), _P(flags_ptr), _P(stream)))


def ps_label_batch_workspace_size(handle, opts: ps_opts | None = None) -> int:
    b = ctypes.c_size_t()
    _check(lib().ps_label_batch_workspace_size(_P(handle), ctypes.byref(opts) if opts is not None else None,
                                               ctypes.byref(b)))
    return b.value


def ps_label_batch(handle, eps, opts, ws_ptr, ws_bytes, label_ptr, sigma_ptr=0, evals_ptr=0, stream=0) -> None:
    _check(lib().ps_label_batch(_P(handle), float(eps), ctypes.byref(opts) if opts is not None else None, _P(ws_ptr),
                                ws_bytes, _P(label_ptr), _P(sigma_ptr), _P(evals_ptr), _P(stream)))


def ps_label_workspace_size(handle, grid: ps_grid, opts: ps_opts | None = None) -> int:
    b = ctypes.c_size_t()
    _check(lib().ps_label_workspace_size(_P(handle), ctypes.byref(grid),
                                         ctypes.byref(opts) if opts is not None else None, ctypes.byref(b)))
    return b.value


def ps_label_grid(handle, grid: ps_grid, eps, opts, ws_ptr, ws_bytes, label_ptr, sigma_ptr=0, evals_ptr=0,
                  stream=0) -> None:
    _check(lib().ps_label_grid(_P(handle), ctypes.byref(grid), float(eps),
                               ctypes.byref(opts) if opts is not None else None, _P(ws_ptr), ws_bytes,
                               _P(label_ptr), _P(sigma_ptr), _P(evals_ptr), _P(stream)))


def ps_contour_seeds_workspace_size(grid: ps_grid) -> int:
    b = ctypes.c_size_t()
    _check(lib().ps_contour_seeds_workspace_size(ctypes.byref(grid), ctypes.byref(b)))
    return b.value


def ps_contour_seeds(grid: ps_grid, sigma_ptr, eps, seeds_ptr, max_seeds, count_ptr, ws_ptr, ws_bytes,
                     stream=0) -> None:
    _check(lib().ps_contour_seeds(ctypes.byref(grid), _P(sigma_ptr), float(eps), _P(seeds_ptr), int(max_seeds),
                                  _P(count_ptr), _P(ws_ptr), ws_bytes, _P(stream)))


def ps_autotune(handle, z_ptr, npts, opts: ps_opts, stream=0) -> ps_opts:
    _check(lib().ps_autotune(_P(handle), _P(z_ptr), npts, ctypes.byref(opts), _P(stream)))
    return opts


def ps_autotune_batch(batch, masks_ptr, opts: ps_opts, stream=0) -> ps_opts:
    _check(lib().ps_autotune_batch(_P(batch), _P(masks_ptr), ctypes.byref(opts), _P(stream)))
    return opts


def ps_plan_cache_clear() -> None:
    lib().ps_plan_cache_clear()


def ps_create_batch(handles, grids) -> int:
    """handles: matrix handles; grids: ps_grid structs (one per matrix).  Returns the batch handle."""
    n = len(handles)
    harr = (_P * n)(*[_P(h) for h in handles])
    garr = (ps_grid * n)(*grids)
    b = _P()
    _check(lib().ps_create_batch(n, harr, garr, ctypes.byref(b)))
    return b.value


def ps_destroy_batch(batch: int) -> None:
    _check(lib().ps_destroy_batch(_P(batch)))


def ps_batch_info(batch: int, nmat: int):
    tot = _I64()
    offs = (_I64 * nmat)()
    _check(lib().ps_batch_info(_P(batch), ctypes.byref(tot), offs))
    return tot.value, list(offs)


def ps_batch_workspace_size(batch: int, opts: ps_opts | None = None) -> int:
    b = ctypes.c_size_t()
    _check(lib().ps_batch_workspace_size(_P(batch), ctypes.byref(opts) if opts is not None else None,
                                         ctypes.byref(b)))
    return b.value


def ps_eval_batch(batch, masks_ptr, opts, ws_ptr, ws_bytes, idx_ptr, counts_ptr, sigma_ptr, info_ptr=0,
                  iters_ptr=0, stream=0) -> None:
    _check(lib().ps_eval_batch(_P(batch), _P(masks_ptr), ctypes.byref(opts) if opts is not None else None,
                               _P(ws_ptr), ws_bytes, _P(idx_ptr), _P(counts_ptr), _P(sigma_ptr), _P(info_ptr),
                               _P(iters_ptr), _P(stream)))


def ps_mask_opts_default(**kw) -> ps_mask_opts:
    o = ps_mask_opts()
    lib().ps_mask_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def ps_mlp_create(params_ptr, flags=0, stream=0) -> int:
    h = _P()
    _check(lib().ps_mlp_create(_P(params_ptr), flags, ctypes.byref(h), _P(stream)))
    return h.value


def ps_mlp_destroy(handle) -> None:
    _check(lib().ps_mlp_destroy(_P(handle)))


def ps_mask_workspace_size(grid, opts) -> int:
    b = ctypes.c_size_t()
    _check(lib().ps_mask_workspace_size(ctypes.byref(grid) if grid is not None else None,
                                        ctypes.byref(opts) if opts is not None else None, ctypes.byref(b)))
    return b.value


def _gfeat(gfeat):
    g = (ctypes.c_double * PS_MLP_NGLOBAL)(*[float(v) for v in gfeat])
    return g


def ps_mlp_prob(handle, gfeat, eig_ptr, neig, z_ptr, npts, ws_ptr, ws_bytes, prob_ptr, stream=0) -> None:
    if len(gfeat) != PS_MLP_NGLOBAL:
        raise ValueError("gfeat needs %d values" % PS_MLP_NGLOBAL)
    _check(lib().ps_mlp_prob(_P(handle), _gfeat(gfeat), _P(eig_ptr), neig, _P(z_ptr), npts, _P(ws_ptr), ws_bytes,
                             _P(prob_ptr), _P(stream)))


def ps_mask_predict(handle, grid: ps_grid, gfeat, eig_ptr, neig, opts, ws_ptr, ws_bytes, mask_ptr, prob_ptr=0,
                    coarse_ptr=0, tau_coarse_ptr=0, evals_ptr=0, stream=0) -> None:
    if len(gfeat) != PS_MLP_NGLOBAL:
        raise ValueError("gfeat needs %d values" % PS_MLP_NGLOBAL)
    _check(lib().ps_mask_predict(_P(handle), ctypes.byref(grid), _gfeat(gfeat), _P(eig_ptr), neig,
                                 ctypes.byref(opts) if opts is not None else None, _P(ws_ptr), ws_bytes,
                                 _P(mask_ptr), _P(prob_ptr), _P(coarse_ptr), _P(tau_coarse_ptr), _P(evals_ptr),
                                 _P(stream)))


def ps_mask_batch_workspace_size(nmat, grid, opts) -> int:
    b = ctypes.c_size_t()
    _check(lib().ps_mask_batch_workspace_size(int(nmat), ctypes.byref(grid),
                                              ctypes.byref(opts) if opts is not None else None, ctypes.byref(b)))
    return b.value


def ps_mask_predict_batch(handle, nmat, grid: ps_grid, gfeat, eig_ptr, eig_off, opts, ws_ptr, ws_bytes, mask_ptr,
                          prob_ptr=0, coarse_ptr=0, tau_coarse_ptr=0, evals_ptr=0, stream=0) -> None:
    """gfeat: nmat * 30 floats (flat or nested); eig_off: nmat + 1 integers (host)."""
    import numpy as _np
    gf = _np.ascontiguousarray(_np.asarray(gfeat, dtype=_np.float64).ravel())
    off = _np.ascontiguousarray(_np.asarray(eig_off, dtype=_np.int64).ravel())
    if gf.size != PS_MLP_NGLOBAL * nmat or off.size != nmat + 1:
        raise ValueError("gfeat needs nmat * %d values and eig_off nmat + 1" % PS_MLP_NGLOBAL)
    _check(lib().ps_mask_predict_batch(_P(handle), int(nmat), ctypes.byref(grid),
                                       gf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _P(eig_ptr),
                                       off.ctypes.data_as(ctypes.POINTER(_I64)),
                                       ctypes.byref(opts) if opts is not None else None, _P(ws_ptr), ws_bytes,
                                       _P(mask_ptr), _P(prob_ptr), _P(coarse_ptr), _P(tau_coarse_ptr), _P(evals_ptr),
                                       _P(stream)))


def ps_mask_calibrate_workspace_size(nval, ntau) -> int:
    b = ctypes.c_size_t()
    _check(lib().ps_mask_calibrate_workspace_size(int(nval), int(ntau), ctypes.byref(b)))
    return b.value


def ps_mask_calibrate(nval, grid: ps_grid, prob_ptr, label_ptr, taus, pred_dilate, label_dilate, median_min, p10_min,
                      ws_ptr, ws_bytes, index_ptr, recall_ptr=0, median_ptr=0, p10_ptr=0, stream=0) -> None:
    t = (ctypes.c_double * max(len(taus), 1))(*[float(v) for v in taus])
    _check(lib().ps_mask_calibrate(int(nval), ctypes.byref(grid), _P(prob_ptr), _P(label_ptr), t, len(taus),
                                   int(pred_dilate), int(label_dilate), float(median_min), float(p10_min),
                                   _P(ws_ptr), ws_bytes, _P(index_ptr), _P(recall_ptr), _P(median_ptr),
                                   _P(p10_ptr), _P(stream)))


def header_symbols():
    """Names of the functions declared in include/ps.h."""
    import re
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ps_[a-z_0-9]+)\s*\(", text)) - {"ps_c128"})
