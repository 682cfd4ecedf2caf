"""CPU-side checks of the C ABI library: it loads, exports every symbol declared in
include/ps.h, and validates arguments on the host before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2605_04550_amd as P


def _lib():
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libps.so not built")
    return P.lib()


def test_library_exports_every_header_symbol():
    L = _lib()
    names = P.header_symbols()
    assert len(names) >= 11
    for name in names:
        assert hasattr(L, name), name
    # the binding exposes every entry point under the same name
    for name in names:
        assert hasattr(P, name), name


def test_header_documents_each_entry_point():
    text = open(P.HEADER).read()
    for name in P.header_symbols():
        # each declaration is preceded by a comment block naming it or grouped with one
        assert re.search(r"\b%s\b" % name, text)


def test_version_and_defaults():
    _lib()
    assert "gfx950" in P.ps_version()
    o = P.ps_opts_default()
    assert o.tol_norm == 1e-10 and o.tol_rel == 1e-8 and o.max_iter == 3000 and o.want_vectors == 0


def _gb(n, kl, ku, fill=1.0):
    return np.full((n, kl + ku + 1), fill, dtype=np.complex128)


def test_create_rejects_bad_arguments_before_any_device_call():
    _lib()
    ab = _gb(8, 1, 1)
    with pytest.raises(P.PsError) as e:
        P.ps_create_banded(ab.ctypes.data, 3, 0, 1, 1)
    assert e.value.status == P.PS_ERR_INVALID
    with pytest.raises(P.PsError) as e:
        P.ps_create_banded(ab.ctypes.data, 3, 8, 1, 8)
    assert e.value.status == P.PS_ERR_INVALID
    with pytest.raises(P.PsError) as e:
        P.ps_create_banded(ab.ctypes.data, 2, 8, 1, 1)          # ldab < kl + ku + 1
    assert e.value.status == P.PS_ERR_INVALID
    with pytest.raises(P.PsError) as e:
        P.ps_create_banded(0, 3, 8, 1, 1)
    assert e.value.status == P.PS_ERR_INVALID
    big = _gb(65, 5, 1)               # kl > 4 is taken as dense, up to n = 64
    with pytest.raises(P.PsError) as e:
        P.ps_create_banded(big.ctypes.data, 7, 65, 5, 1)
    assert e.value.status == P.PS_ERR_UNSUPPORTED
    wide = _gb(64, 5, 1)              # accepted: fails later only for lack of a GPU
    try:
        P.ps_create_banded(wide.ctypes.data, 7, 64, 5, 1)
    except P.PsError as e:
        assert e.status == P.PS_ERR_HIP
    bad = _gb(8, 1, 1)
    bad[3, 1] = np.nan
    with pytest.raises(P.PsError) as e:
        P.ps_create_banded(bad.ctypes.data, 3, 8, 1, 1)
    assert e.value.status == P.PS_ERR_NONFINITE
    assert "non-finite" in P.ps_last_error()
    # NaN in a slot outside the matrix is ignored (not part of A): fails later only for lack of a GPU
    pad = _gb(8, 1, 1)
    pad[0, 0] = np.nan          # ab[j=0, ku + i - j = 0] -> i = -1: outside
    try:
        P.ps_create_banded(pad.ctypes.data, 3, 8, 1, 1)
    except P.PsError as e:
        assert e.status == P.PS_ERR_HIP


def test_null_handle_errors():
    _lib()
    with pytest.raises(P.PsError) as e:
        P.ps_workspace_size(0, 10)
    assert e.value.status == P.PS_ERR_INVALID
    P.ps_destroy(0)   # NULL is accepted
    with pytest.raises(P.PsError):
        P.ps_matrix_info(0)


def test_contour_seed_and_batch_argument_checks():
    """Argument validation of entry points that need no matrix, before any device call."""
    _lib()
    g = P.ps_grid(-1.0, 1.0, -1.0, 1.0, 5, 4)
    need = P.ps_contour_seeds_workspace_size(g)
    assert need >= 256 + 8
    bad = P.ps_grid(-1.0, 1.0, -1.0, 1.0, 0, 4)
    with pytest.raises(P.PsError) as e:
        P.ps_contour_seeds_workspace_size(bad)
    assert e.value.status == P.PS_ERR_INVALID
    nan = P.ps_grid(float("nan"), 1.0, -1.0, 1.0, 5, 4)
    with pytest.raises(P.PsError) as e:
        P.ps_contour_seeds_workspace_size(nan)
    assert e.value.status == P.PS_ERR_NONFINITE
    fake = 1 << 20       # never dereferenced: every call below fails validation first
    for eps in (0.0, -1.0, float("inf")):
        with pytest.raises(P.PsError) as e:
            P.ps_contour_seeds(g, fake, eps, fake, 10, fake, fake, need)
        assert e.value.status == P.PS_ERR_INVALID
    with pytest.raises(P.PsError) as e:            # missing sigma
        P.ps_contour_seeds(g, 0, 1e-3, fake, 10, fake, fake, need)
    assert e.value.status == P.PS_ERR_INVALID
    with pytest.raises(P.PsError) as e:            # seeds NULL with capacity
        P.ps_contour_seeds(g, fake, 1e-3, 0, 10, fake, fake, need)
    assert e.value.status == P.PS_ERR_INVALID
    with pytest.raises(P.PsError) as e:            # workspace too small
        P.ps_contour_seeds(g, fake, 1e-3, fake, 10, fake, fake, need - 1)
    assert e.value.status == P.PS_ERR_WORKSPACE
    with pytest.raises(P.PsError) as e:
        P.ps_create_batch([], [])
    assert e.value.status == P.PS_ERR_INVALID


def test_label_argument_checks():
    _lib()
    g = P.ps_grid(-1.0, 1.0, -1.0, 1.0, 5, 4)
    fake = 1 << 20
    with pytest.raises(P.PsError) as e:
        P.ps_label_workspace_size(0, g)
    assert e.value.status == P.PS_ERR_INVALID
    with pytest.raises(P.PsError) as e:
        P.ps_label_grid(0, g, 0.01, None, fake, 1 << 30, fake)
    assert e.value.status == P.PS_ERR_INVALID


def test_trace_argument_checks():
    _lib()
    o = P.ps_opts_default()
    fake = 256
    for bad in ((0.0, 1e-3, 10, 2), (1e-2, 0.0, 10, 2), (1e-2, float("nan"), 10, 2), (1e-2, 1e-3, 0, 2),
                (1e-2, 1e-3, 10, 0)):
        with pytest.raises(P.PsError) as e:
            P.ps_trace_contour(fake, fake, 4, bad[0], bad[1], bad[2], bad[3], None, o, fake, 1 << 20, fake, fake,
                               fake)
        assert e.value.status == P.PS_ERR_INVALID
    with pytest.raises(P.PsError) as e:
        P.ps_trace_contour(0, fake, 4, 1e-2, 1e-3, 10, 2, None, o, fake, 1 << 20, fake, fake, fake)
    assert e.value.status == P.PS_ERR_INVALID


def test_mask_argument_checks():
    """ps_mlp_create / ps_mlp_prob / ps_mask_predict reject bad arguments before any device call."""
    _lib()
    fake = 256
    params = np.zeros(P.PS_MLP_NPARAM, dtype=np.float32)
    params[123] = np.nan
    with pytest.raises(P.PsError) as e:
        P.ps_mlp_create(params.ctypes.data, 0, 0)
    assert e.value.status == P.PS_ERR_NONFINITE
    with pytest.raises(P.PsError) as e:
        P.ps_mlp_create(0, 0, 0)
    assert e.value.status == P.PS_ERR_INVALID
    with pytest.raises(P.PsError) as e:
        P.ps_mlp_create(params.ctypes.data, 4, 0)               # unknown flag
    assert e.value.status == P.PS_ERR_INVALID
    g = P.ps_grid(-4, 4, -4, 4, 100, 100)
    for bad in (dict(stride=0), dict(stride=33), dict(dilate=4), dict(dilate=0), dict(dilate=33),
                dict(coarse_q=1.5), dict(coarse_q=float("nan")), dict(tau=0.0), dict(tau=1.5)):
        o = P.ps_mask_opts_default(**bad)
        with pytest.raises(P.PsError) as e:
            P.ps_mask_workspace_size(g, o)
        assert e.value.status == P.PS_ERR_INVALID, bad
        with pytest.raises(P.PsError) as e:
            P.ps_mask_predict(fake, g, [0.0] * 30, fake, 4, o, fake, 1 << 20, fake)
        assert e.value.status == P.PS_ERR_INVALID, bad
    # workspace: header + coarse map + probability map, each rounded to 256 bytes
    assert P.ps_mask_workspace_size(None, None) == 1024
    assert P.ps_mask_workspace_size(g, None) == 1024 + 2560 + 40192
    o = P.ps_mask_opts_default()
    with pytest.raises(P.PsError) as e:                          # NULL network
        P.ps_mask_predict(0, g, [0.0] * 30, fake, 4, o, fake, 1 << 20, fake)
    assert e.value.status == P.PS_ERR_INVALID
    with pytest.raises(P.PsError) as e:                          # empty spectrum
        P.ps_mask_predict(fake, g, [0.0] * 30, fake, 0, o, fake, 1 << 20, fake)
    assert e.value.status == P.PS_ERR_INVALID
    with pytest.raises(P.PsError) as e:                          # non-finite global feature
        P.ps_mask_predict(fake, g, [0.0] * 29 + [float("inf")], fake, 4, o, fake, 1 << 20, fake)
    assert e.value.status == P.PS_ERR_NONFINITE
    with pytest.raises(P.PsError) as e:                          # workspace too small
        P.ps_mask_predict(fake, g, [0.0] * 30, fake, 4, o, fake, 1000, fake)
    assert e.value.status == P.PS_ERR_WORKSPACE
    with pytest.raises(P.PsError) as e:                          # mask output missing
        P.ps_mask_predict(fake, g, [0.0] * 30, fake, 4, o, fake, 1 << 20, 0)
    assert e.value.status == P.PS_ERR_INVALID
    with pytest.raises(P.PsError) as e:
        P.ps_mlp_prob(fake, [0.0] * 30, fake, 4, fake, -1, fake, 1024, fake)
    assert e.value.status == P.PS_ERR_INVALID
    with pytest.raises(P.PsError) as e:
        P.ps_mlp_prob(fake, [0.0] * 30, fake, 4, fake, 8, fake, 512, fake)
    assert e.value.status == P.PS_ERR_WORKSPACE


def test_mask_batch_argument_checks():
    _lib()
    fake = 256
    g = P.ps_grid(-4, 4, -4, 4, 100, 100)
    o = P.ps_mask_opts_default()
    gf = np.zeros((3, 30))
    off = np.array([0, 4, 8, 12])
    for nmat in (0, 70000):
        with pytest.raises(P.PsError) as e:
            P.ps_mask_batch_workspace_size(nmat, g, o)
        assert e.value.status == P.PS_ERR_INVALID
    # headers 3 * 1024, gfeat 720 -> 768, offsets 32 -> 256, coarse 3 * 625 * 4 -> 7680, prob 120000
    assert P.ps_mask_batch_workspace_size(3, g, o) == 3072 + 768 + 256 + 7680 + 120064
    bad_off = [np.array([1, 4, 8, 12]), np.array([0, 4, 4, 12]), np.array([0, 4, 8, 7])]
    for b in bad_off:
        with pytest.raises(P.PsError) as e:
            P.ps_mask_predict_batch(fake, 3, g, gf, fake, b, o, fake, 1 << 30, fake)
        assert e.value.status == P.PS_ERR_INVALID, b
    gbad = gf.copy()
    gbad[2, 7] = np.nan
    with pytest.raises(P.PsError) as e:
        P.ps_mask_predict_batch(fake, 3, g, gbad, fake, off, o, fake, 1 << 30, fake)
    assert e.value.status == P.PS_ERR_NONFINITE
    with pytest.raises(P.PsError) as e:
        P.ps_mask_predict_batch(fake, 3, g, gf, fake, off, o, fake, 1000, fake)
    assert e.value.status == P.PS_ERR_WORKSPACE
    with pytest.raises(P.PsError) as e:
        P.ps_mask_predict_batch(0, 3, g, gf, fake, off, o, fake, 1 << 30, fake)
    assert e.value.status == P.PS_ERR_INVALID
    with pytest.raises(ValueError):
        P.ps_mask_predict_batch(fake, 3, g, gf[:2], fake, off, o, fake, 1 << 30, fake)


def test_mask_calibrate_argument_checks():
    _lib()
    fake = 256
    g = P.ps_grid(-4, 4, -4, 4, 100, 100)
    taus = [0.05, 0.1, 0.2]
    assert P.ps_mask_calibrate_workspace_size(30, 90) == 30 * 91 * 8 // 256 * 256 + 256 * ((30 * 91 * 8) % 256 > 0)
    for nval, ntau in ((0, 3), (257, 3), (3, 0), (3, 129)):
        with pytest.raises(P.PsError) as e:
            P.ps_mask_calibrate_workspace_size(nval, ntau)
        assert e.value.status == P.PS_ERR_INVALID
    bad = [dict(taus=[0.1, 0.1]), dict(taus=[0.2, 0.1]), dict(pred_dilate=4), dict(label_dilate=0),
           dict(index=0), dict(prob=0)]
    for b in bad:
        kw = dict(taus=taus, pred_dilate=5, label_dilate=3, index=fake, prob=fake)
        kw.update(b)
        with pytest.raises(P.PsError) as e:
            P.ps_mask_calibrate(3, g, kw["prob"], fake, kw["taus"], kw["pred_dilate"], kw["label_dilate"], 0.9, 0.75,
                                fake, 1 << 20, kw["index"])
        assert e.value.status == P.PS_ERR_INVALID, b
    with pytest.raises(P.PsError) as e:
        P.ps_mask_calibrate(3, g, fake, fake, [0.1, float("nan")], 5, 3, 0.9, 0.75, fake, 1 << 20, fake)
    assert e.value.status == P.PS_ERR_NONFINITE
    with pytest.raises(P.PsError) as e:
        P.ps_mask_calibrate(3, g, fake, fake, taus, 5, 3, 0.9, 0.75, fake, 16, fake)
    assert e.value.status == P.PS_ERR_WORKSPACE
