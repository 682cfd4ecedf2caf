"""Torch-facing helpers over the C ABI (device memory and streams from torch, compute in HIP).

* ``BandedMatrix``   -- owns a ``ps_matrix`` handle (ps_create_banded / ps_destroy).
* ``sigma_min``      -- ps_eval_points on a complex128 CUDA tensor of shifts.
* ``eval_grid``      -- ps_eval_grid on the grid of Sec. 2.1, optionally restricted by a mask (Sec. 4).
* ``SigmaMin``       -- torch.autograd.Function: forward = ps_eval_points with vectors,
                        backward = ps_backward (gradients w.r.t. the shifts and the band).
* ``newton_contour`` -- Newton steps moving points onto the level curve sigma_min = eps.
* ``MaskNet``        -- the classifier of Sec. 3.2 (ps_mlp_create): ``prob`` (ps_mlp_prob) and
                        ``predict`` (ps_mask_predict, the hierarchical prediction of Sec. 3.5).
* ``calibrate_tau``  -- ps_mask_calibrate, the threshold calibration of Sec. 3.6.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import (PS_DEVICE_PTR, PS_REAL_A, ps_autotune, ps_autotune_batch, ps_backward, ps_backward_workspace_size, ps_batch_info,
               ps_batch_workspace_size, ps_create_banded, ps_create_batch, ps_destroy, ps_destroy_batch,
               ps_eval_batch, ps_eval_grid, ps_eval_points, ps_grid, ps_matrix_info, ps_newton_contour,
               ps_newton_workspace_size, ps_opts_default, ps_workspace_size, ps_contour_seeds,
               ps_contour_seeds_workspace_size, ps_label_grid, ps_label_workspace_size, ps_label_batch,
               ps_label_batch_workspace_size, ps_trace_contour, ps_trace_workspace_size, ps_mask_opts_default,
               ps_mlp_create, ps_mlp_destroy, ps_mask_workspace_size, ps_mlp_prob, ps_mask_predict,
               ps_mask_batch_workspace_size, ps_mask_predict_batch, ps_mask_calibrate,
               ps_mask_calibrate_workspace_size, PS_MLP_NPARAM)

__all__ = ["BandedMatrix", "BandedBatch", "sigma_min", "eval_grid", "SigmaMin", "newton_contour", "make_opts",
           "MaskNet", "calibrate_tau"]


def _stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def make_opts(tol_norm=1e-10, tol_rel=1e-8, max_iter=3000, want_vectors=False, slots=0, check_shift=0,
              bisect=True, lanes=0, tests=0):
    return ps_opts_default(tol_norm=tol_norm, tol_rel=tol_rel, max_iter=max_iter,
                           want_vectors=int(bool(want_vectors)), slots=int(slots), check_shift=int(check_shift),
                           bisect=0 if bisect else -1, lanes=int(lanes), tests=int(tests))


class BandedMatrix:
    """A banded matrix registered with the library (GB storage, see include/ps.h)."""

    def __init__(self, ab, n: int, kl: int, ku: int, real: bool = False):
        if isinstance(ab, torch.Tensor):
            t = ab.detach().to(torch.complex128).contiguous()
            flags = PS_DEVICE_PTR if t.is_cuda else 0
            ptr = t.data_ptr()
            keep = t
        else:
            keep = np.ascontiguousarray(ab, dtype=np.complex128)
            flags = 0
            ptr = keep.ctypes.data
        if real:
            flags |= PS_REAL_A
        self.handle = ps_create_banded(ptr, kl + ku + 1, n, kl, ku, flags, _stream_handle() if flags & 1 else 0)
        # the band the handle holds, kept for SigmaMin's check that its band argument still is it
        self.band = keep.clone() if isinstance(keep, torch.Tensor) else torch.from_numpy(keep.copy())
        del keep
        self.n, self.kl, self.ku, self.fro = ps_matrix_info(self.handle)
        self.real = real

    @classmethod
    def from_band(cls, band):
        return cls(band.ab, band.n, band.kl, band.ku, real=bool(getattr(band, "real", False)))

    def close(self):
        if getattr(self, "handle", None):
            ps_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BandedBatch:
    """Many registered matrices, each with its own grid, evaluated by one ps_eval_batch call."""

    def __init__(self, mats, grids):
        self.mats = list(mats)
        self.grids = [ps_grid(float(g.a), float(g.b), float(g.c), float(g.d), int(g.nx), int(g.ny)) for g in grids]
        self.handle = ps_create_batch([m.handle for m in self.mats], self.grids)
        self.total, self.offsets = ps_batch_info(self.handle, len(self.mats))

    def close(self):
        if getattr(self, "handle", None):
            ps_destroy_batch(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _mask_ptr(self, masks, dev, keep):
        """Device address of the mask table (0 for none); tensors it refers to go into keep."""
        nmat = len(self.mats)
        if isinstance(masks, torch.Tensor):
            assert masks.is_cuda and masks.dtype == torch.int64 and masks.numel() == nmat
            keep.append(masks)
            return masks.data_ptr()
        if masks is None:
            return 0
        ptrs = []
        for m, mk in enumerate(masks):
            if mk is None:
                ptrs.append(0)
            else:
                assert mk.is_cuda and mk.dtype == torch.uint8 and mk.numel() == self.grids[m].nx * self.grids[m].ny
                mk = mk.contiguous()
                keep.append(mk)
                ptrs.append(mk.data_ptr())
        parr = torch.tensor(ptrs, dtype=torch.int64, device=dev)
        keep.append(parr)
        return parr.data_ptr()

    def autotune(self, masks=None, *, device=None, stream=None, **kw):
        """ps_autotune_batch with these masks: returns the options (lanes, tests or check_shift set,
        the rest as given by kw) that ran fastest; cached per process."""
        dev = device or torch.device("cuda")
        o = make_opts(**kw)
        keep = []
        mptr = self._mask_ptr(masks, dev, keep)
        ps_autotune_batch(self.handle, mptr, o, _stream_handle(stream))
        return o

    def eval(self, masks=None, *, tol_norm=1e-10, tol_rel=1e-8, max_iter=3000, slots=0, bisect=True,
             device=None, stream=None, workspace: torch.Tensor | None = None, lanes=0, tests=0, check_shift=0,
             opts=None):
        """masks: list of uint8 CUDA tensors [ny, nx] (None entries = full grid) or None, or the device
        table of their addresses (an int64 CUDA tensor from ``mask_table``, which a captured graph needs:
        building the table copies from the host).  opts: a ps_opts (e.g. from ``autotune``) used
        instead of the keyword options.  Returns dict with the concatenated idx, sigma, info, iters,
        and counts [nmat]; matrix m owns offsets[m] onward."""
        dev = device or torch.device("cuda")
        nmat = len(self.mats)
        o = opts if opts is not None else make_opts(tol_norm, tol_rel, max_iter, False, slots, check_shift,
                                                      bisect=bisect, lanes=lanes, tests=tests)
        keep = []
        mptr = self._mask_ptr(masks, dev, keep)
        out = dict(idx=torch.empty(self.total, dtype=torch.int64, device=dev),
                   counts=torch.zeros(nmat, dtype=torch.int64, device=dev),
                   sigma=torch.full((self.total,), float("nan"), dtype=torch.float64, device=dev),
                   info=torch.empty(self.total, dtype=torch.int32, device=dev),
                   iters=torch.empty(self.total, dtype=torch.int32, device=dev),
                   offsets=list(self.offsets))
        need = ps_batch_workspace_size(self.handle, o)
        ws = workspace if workspace is not None else _workspace(need, dev)
        ps_eval_batch(self.handle, mptr, o, ws.data_ptr(), ws.numel(), out["idx"].data_ptr(), out["counts"].data_ptr(),
                      out["sigma"].data_ptr(), out["info"].data_ptr(), out["iters"].data_ptr(), _stream_handle(stream))
        out["_keep"] = keep
        return out

    def mask_table(self, masks, device=None):
        """The device table of mask addresses for ``eval`` (keep the masks alive while it is used)."""
        dev = device or torch.device("cuda")
        ptrs = []
        for m, mk in enumerate(masks):
            if mk is None:
                ptrs.append(0)
            else:
                assert mk.is_cuda and mk.dtype == torch.uint8 and mk.is_contiguous()
                assert mk.numel() == self.grids[m].nx * self.grids[m].ny
                ptrs.append(mk.data_ptr())
        return torch.tensor(ptrs, dtype=torch.int64, device=dev)

    def label(self, eps: float, *, tol_norm=1e-10, tol_rel=1e-8, max_iter=3000, slots=0, bisect=True,
              device=None, stream=None):
        """ps_label_batch: labels (sigma_min <= eps) of every grid point of every matrix, by exclusion
        regions.  Returns dict(label [total] uint8, sigma [total] (-1 where excluded), evals, offsets)."""
        dev = device or torch.device("cuda")
        o = make_opts(tol_norm, tol_rel, max_iter, False, slots, bisect=bisect)
        out = dict(label=torch.empty(self.total, dtype=torch.uint8, device=dev),
                   sigma=torch.empty(self.total, dtype=torch.float64, device=dev),
                   evals=torch.zeros(1, dtype=torch.int64, device=dev), offsets=list(self.offsets))
        ws = _workspace(ps_label_batch_workspace_size(self.handle, o), dev)
        ps_label_batch(self.handle, eps, o, ws.data_ptr(), ws.numel(), out["label"].data_ptr(),
                       out["sigma"].data_ptr(), out["evals"].data_ptr(), _stream_handle(stream))
        return out


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def sigma_min(mat: BandedMatrix, z: torch.Tensor, *, want_vectors=False, tol_norm=1e-10, tol_rel=1e-8,
              max_iter=3000, slots=0, bisect=True, workspace: torch.Tensor | None = None, stream=None, lanes=0,
              tests=0):
    """sigma_min(z_p I - A) for every entry of the complex128 CUDA tensor z.  Returns a dict
    with ``sigma`` (float64), ``info`` and ``iters`` (int32), and ``u``, ``v`` ([npts, n]) if asked."""
    assert z.is_cuda and z.dtype == torch.complex128
    z = z.contiguous()
    npts = z.numel()
    dev = z.device
    o = make_opts(tol_norm, tol_rel, max_iter, want_vectors, slots, bisect=bisect, lanes=lanes, tests=tests)
    out = dict(sigma=torch.empty(npts, dtype=torch.float64, device=dev),
               info=torch.empty(npts, dtype=torch.int32, device=dev),
               iters=torch.empty(npts, dtype=torch.int32, device=dev))
    if want_vectors:
        out["u"] = torch.empty((npts, mat.n), dtype=torch.complex128, device=dev)
        out["v"] = torch.empty((npts, mat.n), dtype=torch.complex128, device=dev)
    if npts == 0:
        return out
    need = ps_workspace_size(mat.handle, npts, o)
    ws = workspace if workspace is not None else _workspace(need, dev)
    ps_eval_points(mat.handle, z.data_ptr(), npts, o, ws.data_ptr(), ws.numel(), out["sigma"].data_ptr(),
                   out["u"].data_ptr() if want_vectors else 0, out["v"].data_ptr() if want_vectors else 0,
                   out["info"].data_ptr(), out["iters"].data_ptr(), _stream_handle(stream))
    return out


def eval_grid(mat: BandedMatrix, grid, mask: torch.Tensor | None = None, *, eps=None, want_vectors=False,
              tol_norm=1e-10, tol_rel=1e-8, max_iter=3000, slots=0, bisect=True, device=None, stream=None,
              workspace: torch.Tensor | None = None, lanes=0, tests=0):
    """sigma_min on the grid (a, b, c, d, nx, ny) of Sec. 2.1, or on the points where ``mask`` (uint8
    [ny, nx] CUDA tensor) is nonzero.  Outputs are compacted: entry p belongs to flat grid index
    ``idx[p]``, for p < ``count``."""
    g = ps_grid(float(grid.a), float(grid.b), float(grid.c), float(grid.d), int(grid.nx), int(grid.ny))
    npts = g.nx * g.ny
    dev = mask.device if mask is not None else (device or torch.device("cuda"))
    o = make_opts(tol_norm, tol_rel, max_iter, want_vectors, slots, bisect=bisect, lanes=lanes, tests=tests)
    out = dict(idx=torch.empty(npts, dtype=torch.int64, device=dev),
               count=torch.zeros(1, dtype=torch.int64, device=dev),
               sigma=torch.empty(npts, dtype=torch.float64, device=dev),
               info=torch.empty(npts, dtype=torch.int32, device=dev),
               iters=torch.empty(npts, dtype=torch.int32, device=dev))
    if eps is not None:
        out["sens"] = torch.empty(npts, dtype=torch.uint8, device=dev)
    if want_vectors:
        out["u"] = torch.empty((npts, mat.n), dtype=torch.complex128, device=dev)
        out["v"] = torch.empty((npts, mat.n), dtype=torch.complex128, device=dev)
    if mask is not None:
        assert mask.is_cuda and mask.dtype == torch.uint8 and mask.numel() == npts
        mask = mask.contiguous()
    need = ps_workspace_size(mat.handle, npts, o)
    ws = workspace if workspace is not None else _workspace(need, dev)
    ps_eval_grid(mat.handle, g, mask.data_ptr() if mask is not None else 0, o, ws.data_ptr(), ws.numel(),
                 out["idx"].data_ptr(), out["count"].data_ptr(), out["sigma"].data_ptr(),
                 out["u"].data_ptr() if want_vectors else 0, out["v"].data_ptr() if want_vectors else 0,
                 out["info"].data_ptr(), out["iters"].data_ptr(), float(eps) if eps is not None else 0.0,
                 out["sens"].data_ptr() if eps is not None else 0, _stream_handle(stream))
    return out


def backward(mat: BandedMatrix, grad_sigma: torch.Tensor, u: torch.Tensor, v: torch.Tensor, want_z=True,
             want_band=True, stream=None):
    """ps_backward: returns (grad_z [npts] complex128, grad_band [n, kl+ku+1] complex128 in GB layout)."""
    npts = grad_sigma.numel()
    dev = grad_sigma.device
    gz = torch.empty(npts, dtype=torch.complex128, device=dev) if want_z else None
    gb = torch.empty((mat.n, mat.kl + mat.ku + 1), dtype=torch.complex128, device=dev) if want_band else None
    need = ps_backward_workspace_size(mat.handle, npts)
    ws = _workspace(need, dev)
    ps_backward(mat.handle, npts, grad_sigma.contiguous().data_ptr(), u.contiguous().data_ptr(),
                v.contiguous().data_ptr(), gz.data_ptr() if gz is not None else 0,
                gb.data_ptr() if gb is not None else 0, ws.data_ptr(), ws.numel(), _stream_handle(stream))
    return gz, gb


class SigmaMin(torch.autograd.Function):
    """sigma = SigmaMin.apply(band, z, mat): band is a complex128 GB tensor [n, kl + ku + 1] of the
    matrix (kl, ku and the real flag come from the handle mat), z the shifts.  sigma and both
    gradients belong to the values band holds at the call: when they differ from the band mat
    was built from (an in-place edit, another tensor), a handle is built from band for the call.
    Gradients follow the conjugate-Wirtinger convention torch uses for complex tensors."""

    @staticmethod
    def forward(ctx, band, z, mat, tol_norm=1e-10, tol_rel=1e-8):
        b = band.detach()
        if tuple(b.shape) != (mat.n, mat.kl + mat.ku + 1):
            raise ValueError("band has shape %s; the handle's matrix needs (%d, %d)"
                             % (tuple(b.shape), mat.n, mat.kl + mat.ku + 1))
        if not torch.equal(b.to(mat.band.device, torch.complex128), mat.band):
            real = mat.real and not bool(torch.any(b.imag != 0))   # an edit may leave A complex
            mat = BandedMatrix(b, mat.n, mat.kl, mat.ku, real=real)
        r = sigma_min(mat, z.detach(), want_vectors=True, tol_norm=tol_norm, tol_rel=tol_rel)
        ctx.mat = mat
        ctx.save_for_backward(r["u"], r["v"])
        ctx.band_shape = band.shape
        return r["sigma"]

    @staticmethod
    def backward(ctx, g):
        u, v = ctx.saved_tensors
        mat = ctx.mat
        gz, gb = backward(mat, g.to(torch.float64), u, v, want_z=ctx.needs_input_grad[1],
                          want_band=ctx.needs_input_grad[0])
        return gb, gz, None, None, None


def newton_contour(mat: BandedMatrix, z0: torch.Tensor, eps: float, steps: int = 3, tol_rel=1e-12, tol_norm=1e-14,
                   stream=None):
    """ps_newton_contour: `steps` Newton steps on ln(sigma_min/eps) along g = conj(u^H v), all on the GPU.
    Returns the refined points and sigma_min there."""
    z = z0.detach().to(torch.complex128).contiguous().clone()
    npts = z.numel()
    dev = z.device
    o = make_opts(tol_norm, tol_rel, 3000, True, 0)
    sig = torch.empty(npts, dtype=torch.float64, device=dev)
    info = torch.empty(npts, dtype=torch.int32, device=dev)
    ws = _workspace(ps_newton_workspace_size(mat.handle, npts, o), dev)
    ps_newton_contour(mat.handle, z.data_ptr(), npts, eps, steps, o, ws.data_ptr(), ws.numel(), sig.data_ptr(),
                      info.data_ptr(), _stream_handle(stream))
    return z, sig


def trace_contour(mat: BandedMatrix, seeds: torch.Tensor, eps: float, h: float, max_points: int,
                  newton_steps: int = 2, box=None, tol_rel=1e-8, tol_norm=1e-10, stream=None):
    """ps_trace_contour: follow the eps-level curve from each seed (tangent step of length h,
    then Newton corrections).  box: (a, b, c, d) or None.  Returns dict(points [nseed,
    max_points] complex128, count [nseed] int32, flags [nseed] int32, PS_TRACE_* bits)."""
    z = seeds.detach().to(torch.complex128).contiguous()
    m = z.numel()
    dev = z.device
    o = make_opts(tol_norm, tol_rel, 3000, True, 0)
    pts = torch.zeros((m, max_points), dtype=torch.complex128, device=dev)
    count = torch.zeros(m, dtype=torch.int32, device=dev)
    flags = torch.zeros(m, dtype=torch.int32, device=dev)
    g = None if box is None else ps_grid(float(box[0]), float(box[1]), float(box[2]), float(box[3]), 1, 1)
    ws = _workspace(ps_trace_workspace_size(mat.handle, m, o), dev)
    ps_trace_contour(mat.handle, z.data_ptr(), m, eps, h, max_points, newton_steps, g, o, ws.data_ptr(), ws.numel(),
                     pts.data_ptr(), count.data_ptr(), flags.data_ptr(), _stream_handle(stream))
    return dict(points=pts, count=count, flags=flags)


def contour_seeds(grid, sigma: torch.Tensor, eps: float, max_seeds: int | None = None, stream=None):
    """ps_contour_seeds: points on the eps-level curve from sign changes of sigma - eps along the
    edges of the grid whose full-grid sigma (row-major [ny * nx], on the device) is given.
    Returns (seeds [min(count, max_seeds)] complex128, count)."""
    g = ps_grid(float(grid.a), float(grid.b), float(grid.c), float(grid.d), int(grid.nx), int(grid.ny))
    dev = sigma.device
    assert sigma.dtype == torch.float64 and sigma.numel() == g.nx * g.ny
    if max_seeds is None:
        max_seeds = g.ny * (g.nx - 1) + (g.ny - 1) * g.nx
    seeds = torch.empty(max(int(max_seeds), 1), dtype=torch.complex128, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = _workspace(ps_contour_seeds_workspace_size(g), dev)
    ps_contour_seeds(g, sigma.contiguous().data_ptr(), eps, seeds.data_ptr(), int(max_seeds), count.data_ptr(),
                     ws.data_ptr(), ws.numel(), _stream_handle(stream))
    c = int(count.item())
    return seeds[:min(c, int(max_seeds))], c


def label_grid(mat: BandedMatrix, grid, eps: float, *, tol_norm=1e-10, tol_rel=1e-8, max_iter=3000, slots=0,
               bisect=True, device=None, stream=None):
    """ps_label_grid: the sensitive zone S_eps on the whole grid (label 1 iff sigma_min <= eps),
    evaluating sigma_min only outside the exclusion disks of points already evaluated.
    Returns dict(label [ny, nx] uint8, sigma [ny, nx] float64 (-1 where excluded), evals)."""
    g = ps_grid(float(grid.a), float(grid.b), float(grid.c), float(grid.d), int(grid.nx), int(grid.ny))
    dev = device or torch.device("cuda")
    o = make_opts(tol_norm, tol_rel, max_iter, False, slots, bisect=bisect)
    label = torch.empty((g.ny, g.nx), dtype=torch.uint8, device=dev)
    sigma = torch.empty((g.ny, g.nx), dtype=torch.float64, device=dev)
    evals = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = _workspace(ps_label_workspace_size(mat.handle, g, o), dev)
    ps_label_grid(mat.handle, g, eps, o, ws.data_ptr(), ws.numel(), label.data_ptr(), sigma.data_ptr(),
                  evals.data_ptr(), _stream_handle(stream))
    return dict(label=label, sigma=sigma, evals=evals)


def autotune(mat: BandedMatrix, z: torch.Tensor, **kw):
    """ps_autotune on the shifts z: returns the options that ran fastest (lanes and tests for sigma-only
    calls that bisect, else slots and check_shift; the rest as given by kw); cached per process."""
    o = make_opts(**kw)
    ps_autotune(mat.handle, z.contiguous().data_ptr(), z.numel(), o, _stream_handle())
    return o


def calibrate_tau(grid, prob: torch.Tensor, labels: torch.Tensor, taus=None, *, pred_dilate=5, label_dilate=3,
                  median_min=0.90, p10_min=0.75, stream=None):
    """ps_mask_calibrate on probability maps prob [nval, ny, nx] (float32) and labels [nval, ny, nx]
    (uint8), both CUDA tensors.  taus defaults to 0.05, 0.06, ..., 0.94.  Returns dict(index
    (smallest qualifying candidate, -1 if none), index_max, taus, recall [nval, ntau],
    median [ntau], p10 [ntau])."""
    if taus is None:
        taus = [round(0.05 + 0.01 * k, 2) for k in range(90)]
    g = ps_grid(float(grid.a), float(grid.b), float(grid.c), float(grid.d), int(grid.nx), int(grid.ny))
    nval = prob.shape[0]
    assert prob.dtype == torch.float32 and labels.dtype == torch.uint8 and prob.numel() == labels.numel()
    assert prob.numel() == nval * g.nx * g.ny
    dev = prob.device
    prob = prob.contiguous()
    labels = labels.contiguous()
    ntau = len(taus)
    idx = torch.empty(2, dtype=torch.int32, device=dev)
    recall = torch.empty((nval, ntau), dtype=torch.float64, device=dev)
    med = torch.empty(ntau, dtype=torch.float64, device=dev)
    p10 = torch.empty(ntau, dtype=torch.float64, device=dev)
    ws = _workspace(ps_mask_calibrate_workspace_size(nval, ntau), dev)
    ps_mask_calibrate(nval, g, prob.data_ptr(), labels.data_ptr(), taus, pred_dilate, label_dilate, median_min,
                      p10_min, ws.data_ptr(), ws.numel(), idx.data_ptr(), recall.data_ptr(), med.data_ptr(),
                      p10.data_ptr(), _stream_handle(stream))
    i = idx.cpu().tolist()
    return dict(index=i[0], index_max=i[1], taus=list(taus), recall=recall, median=med, p10=p10)


class MaskNet:
    """The classifier of Sec. 3.2 registered with the library (ps_mlp_create / ps_mlp_destroy).

    params: PS_MLP_NPARAM float32 values in the layout of include/ps.h (numpy array or CUDA
    tensor)."""

    def __init__(self, params):
        if isinstance(params, torch.Tensor):
            t = params.detach().to(torch.float32).contiguous()
            assert t.numel() == PS_MLP_NPARAM
            self.handle = ps_mlp_create(t.data_ptr(), PS_DEVICE_PTR if t.is_cuda else 0,
                                        _stream_handle() if t.is_cuda else 0)
        else:
            keep = np.ascontiguousarray(params, dtype=np.float32).ravel()
            assert keep.size == PS_MLP_NPARAM
            self.handle = ps_mlp_create(keep.ctypes.data, 0, _stream_handle())

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                ps_mlp_destroy(h)
            except Exception:
                pass
            self.handle = None

    def prob(self, gfeat, eig: torch.Tensor, z: torch.Tensor, stream=None) -> torch.Tensor:
        """ps_mlp_prob: p(z, A) at the points z (complex128 CUDA tensor); eig: the eigenvalues of A
        (complex128 CUDA tensor); gfeat: the 30 global features (host floats)."""
        eig = eig.contiguous()
        z = z.contiguous()
        prob = torch.empty(z.numel(), dtype=torch.float32, device=z.device)
        ws = _workspace(ps_mask_workspace_size(None, None), z.device)
        ps_mlp_prob(self.handle, list(gfeat), eig.data_ptr(), eig.numel(), z.data_ptr(), z.numel(), ws.data_ptr(),
                    ws.numel(), prob.data_ptr(), _stream_handle(stream))
        return prob

    def predict(self, grid, gfeat, eig: torch.Tensor, *, tau=0.05, stride=4, dilate=5, coarse_q=0.8, stream=None):
        """ps_mask_predict: the predicted region R on the grid (Sec. 3.5 / Sec. 4).  Returns
        dict(mask [ny, nx] uint8, prob [ny, nx] float32, coarse [cy, cx] float32,
        tau_coarse (0-d float64 tensor), evals (1-element int64 tensor))."""
        g = ps_grid(float(grid.a), float(grid.b), float(grid.c), float(grid.d), int(grid.nx), int(grid.ny))
        o = ps_mask_opts_default(stride=int(stride), dilate=int(dilate), coarse_q=float(coarse_q), tau=float(tau))
        eig = eig.contiguous()
        dev = eig.device
        cy, cx = (g.ny + o.stride - 1) // o.stride, (g.nx + o.stride - 1) // o.stride
        mask = torch.empty((g.ny, g.nx), dtype=torch.uint8, device=dev)
        prob = torch.empty((g.ny, g.nx), dtype=torch.float32, device=dev)
        coarse = torch.empty((cy, cx), dtype=torch.float32, device=dev)
        tau_c = torch.empty((), dtype=torch.float64, device=dev)
        evals = torch.empty(1, dtype=torch.int64, device=dev)
        ws = _workspace(ps_mask_workspace_size(g, o), dev)
        ps_mask_predict(self.handle, g, list(gfeat), eig.data_ptr(), eig.numel(), o, ws.data_ptr(), ws.numel(),
                        mask.data_ptr(), prob.data_ptr(), coarse.data_ptr(), tau_c.data_ptr(), evals.data_ptr(),
                        _stream_handle(stream))
        return dict(mask=mask, prob=prob, coarse=coarse, tau_coarse=tau_c, evals=evals)

    def predict_batch(self, grid, gfeats, eigs, *, tau=0.05, stride=4, dilate=5, coarse_q=0.8, stream=None):
        """ps_mask_predict_batch: ``predict`` for several matrices on one grid in one set of launches.
        gfeats: nmat x 30 host values; eigs: list of complex128 CUDA tensors (one spectrum per matrix).
        Returns the same dict as ``predict`` with a leading matrix axis."""
        g = ps_grid(float(grid.a), float(grid.b), float(grid.c), float(grid.d), int(grid.nx), int(grid.ny))
        o = ps_mask_opts_default(stride=int(stride), dilate=int(dilate), coarse_q=float(coarse_q), tau=float(tau))
        nmat = len(eigs)
        dev = eigs[0].device
        eig = torch.cat([e.reshape(-1) for e in eigs]).contiguous()
        off = np.concatenate([[0], np.cumsum([e.numel() for e in eigs])]).astype(np.int64)
        cy, cx = (g.ny + o.stride - 1) // o.stride, (g.nx + o.stride - 1) // o.stride
        mask = torch.empty((nmat, g.ny, g.nx), dtype=torch.uint8, device=dev)
        prob = torch.empty((nmat, g.ny, g.nx), dtype=torch.float32, device=dev)
        coarse = torch.empty((nmat, cy, cx), dtype=torch.float32, device=dev)
        tau_c = torch.empty(nmat, dtype=torch.float64, device=dev)
        evals = torch.empty(nmat, dtype=torch.int64, device=dev)
        ws = _workspace(ps_mask_batch_workspace_size(nmat, g, o), dev)
        ps_mask_predict_batch(self.handle, nmat, g, np.asarray(gfeats, dtype=np.float64), eig.data_ptr(), off, o,
                              ws.data_ptr(), ws.numel(), mask.data_ptr(), prob.data_ptr(), coarse.data_ptr(),
                              tau_c.data_ptr(), evals.data_ptr(), _stream_handle(stream))
        return dict(mask=mask, prob=prob, coarse=coarse, tau_coarse=tau_c, evals=evals)
