"""CPU oracle for the mask producer of Sec. 3: the classifier p(z, A), its hierarchical
coarse-to-fine evaluation over a grid, the calibrated threshold and the dilation that turn
it into the restricted set R handed to the sigma_min path.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle``): it shares no code with the GPU
library; the two meet only through the seeded inputs of ``workloads``.  Arithmetic is
float64 throughout (the network's weights are float32 numbers, used exactly).

Contents, each following the passage named in its docstring:
  * ``unpack``             -- the parameter vector split into the layers of Sec. 3.2.
  * ``fourier_features``   -- phi(c) of Sec. 3.2 (Fourier feature encoding), 26 values.
  * ``point_features``     -- g1, g2, g3 of Sec. 3.1, eq. (dist).
  * ``mlp_prob``           -- p(z, A) of Sec. 3.2 (dual-path network), with an optional
                              a-priori bound on the error of a float32 evaluation.
  * ``quantile_linear``    -- the 80th-percentile threshold of Sec. 3.5 (hierarchical
                              prediction), linear interpolation between order statistics.
  * ``hierarchical_mask``  -- Sec. 3.5 and Sec. 4: coarse grid of stride s, refinement of
                              the cells at or above the percentile, threshold tau, square
                              dilation.
  * ``mask_predict``       -- ``hierarchical_mask`` with the network as the probability.
  * ``calibrate_tau``      -- the threshold calibration of Sec. 3.6: recall of the dilated
                              predictions against the dilated labels, the smallest candidate
                              whose median and 10th-percentile recall reach their bounds.
Pins: ``tests/test_oracle_mask_pins.py`` (closed forms, torch.nn layers as an independent
implementation of the network, numpy's quantile, scipy's dilation, brute force).
"""
from __future__ import annotations

import math

import numpy as np

# Layer shapes of Sec. 3.2 (out, in), in the order the parameter vector stores them; each
# layer is its weight matrix W (out x in, row-major, y = W h + b) followed by its bias b.
LAYERS = (
    ("c1", 64, 26),    # coordinate path, on phi(c)
    ("c2", 64, 64),
    ("m1", 128, 33),   # matrix path, on f(z, A) = [f1 .. f30, g1, g2, g3]
    ("m2", 64, 128),
    ("r4", 128, 128),  # on the concatenation [h_c2, h_m2]
    ("r5", 128, 128),  # residual branch: h6 = h4 + SiLU(W5 h4 + b5)
    ("p7", 64, 128),
    ("out", 1, 64),    # logit w^T h7 + b
)
NPARAM = sum(o * i + o for _, o, i in LAYERS)     # 59 841 (the paper's stated layer shapes)
NGLOBAL = 30                                      # f1 .. f30 (Tables matrix, matrixAdd, resolvent)
U32 = 2.0 ** -24                                  # unit roundoff of float32


def unpack(params):
    """Split the flat parameter vector into {name: (W, b)} (float64 copies), Sec. 3.2."""
    p = np.asarray(params, dtype=np.float64).ravel()
    if p.size != NPARAM:
        raise ValueError("expected %d parameters, got %d" % (NPARAM, p.size))
    out, at = {}, 0
    for name, o, i in LAYERS:
        W = p[at:at + o * i].reshape(o, i)
        at += o * i
        b = p[at:at + o].copy()
        at += o
        out[name] = (W, b)
    return out


def fourier_features(x, y):
    """Sec. 3.2, Fourier feature encoding: phi(c) = [c, sin(2c), cos(2c), sin(4c), cos(4c), ...,
    sin(64c), cos(64c)] for c = [x, y], element-wise over c; 2 + 6 * 4 = 26 values per point."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    cols = [x, y]
    for k in range(1, 7):
        f = float(2 ** k)
        cols += [np.sin(f * x), np.sin(f * y), np.cos(f * x), np.cos(f * y)]
    return np.stack(cols, axis=1)


def point_features(z, eig):
    """Sec. 3.1, eq. (dist): g1 = min_i |z - lambda_i|, g2 = |z - lambda*|, g3 = mean_i |z - lambda_i|.

    lambda* is not defined in the paper; it is read as the eigenvalue centroid (the mean of
    the eigenvalues, the point the resolvent features of the same section are taken around)."""
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    eig = np.asarray(eig, dtype=np.complex128).ravel()
    if eig.size == 0:
        raise ValueError("the spectrum is empty")
    d = np.abs(z[:, None] - eig[None, :])
    cent = eig.mean()
    return np.stack([d.min(axis=1), np.abs(z - cent), d.mean(axis=1)], axis=1)


def _silu(x):
    with np.errstate(over="ignore"):
        return x / (1.0 + np.exp(-x))


def _sigmoid(x):
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(-x))


def _gamma(k):
    return k * U32 / (1.0 - k * U32)


def _dsilu(y):
    """d/dy SiLU(y) = s (1 + y (1 - s)), s = sigmoid(y)."""
    s = _sigmoid(y)
    return s * (1.0 + y * (1.0 - s))


def _act_err(y):
    """Relative error allowed for one SiLU / sigmoid evaluation in float32 at argument y:
    exp through exp2 with the argument scaled (|y| u twice), exp2 and the reciprocal to an
    ulp each, two roundings (1 + e, the product)."""
    return (4.0 * (1.0 + np.abs(y)) + 4.0) * U32


def mlp_prob(params, gfeat, eig, z, bound=False):
    """Sec. 3.2: p(z, A) = sigmoid(w^T h7 + b) of the dual-path network, for points z.

    gfeat: the 30 global matrix features f1 .. f30 (computed by the caller); eig: the
    eigenvalues of A (for g1 .. g3).  Coordinates c = [Re z, Im z].

    With bound=True also returns, per point, a bound on |p_float32 - p| for an evaluation in
    float32 arithmetic, by first-order forward error analysis: every rounding site s (an input
    rounded to float32, a dense layer's output accumulated in float32 in any order, a SiLU or
    sigmoid evaluation, the residual sum) contributes |dp/ds| times its local error bound
    (gamma_{K+1} (|W| |h| + |b|) for a dense output, ``_act_err`` |a| for an activation, u |x|
    for an input or a sum); dp/ds comes from the network's exact derivatives (a backward
    pass).  The first-order sum is doubled to cover the higher-order terms."""
    L = unpack(params)
    gfeat = np.asarray(gfeat, dtype=np.float64).ravel()
    if gfeat.size != NGLOBAL:
        raise ValueError("expected %d global features" % NGLOBAL)
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    m = z.size
    phi = fourier_features(z.real, z.imag)                                  # (m, 26)
    feat = np.concatenate([np.broadcast_to(gfeat, (m, NGLOBAL)), point_features(z, eig)], axis=1)

    def dense(name, h):
        W, b = L[name]
        return h @ W.T + b

    yc1 = dense("c1", phi)
    hc1 = _silu(yc1)                                                        # h_c^(1)
    yc2 = dense("c2", hc1)
    hc2 = _silu(yc2)                                                        # h_c^(2)
    ym1 = dense("m1", feat)
    hm1 = _silu(ym1)                                                        # h_m^(1)
    ym2 = dense("m2", hm1)
    hm2 = _silu(ym2)                                                        # h_m^(2)
    h3 = np.concatenate([hc2, hm2], axis=1)                                 # [h_c^(2), h_m^(2)]
    y4 = dense("r4", h3)
    h4 = _silu(y4)
    y5 = dense("r5", h4)
    h5 = _silu(y5)
    h6 = h4 + h5                                                            # residual connection
    y7 = dense("p7", h6)
    h7 = _silu(y7)
    zl = dense("out", h7)[:, 0]
    p = _sigmoid(zl)
    if not bound:
        return p

    # backward pass: exact sensitivities of p to every intermediate
    def back(name, gy):
        return gy @ L[name][0]

    def local(name, h):
        W, b = L[name]
        return _gamma(W.shape[1] + 1) * (np.abs(h) @ np.abs(W).T + np.abs(b))

    g_zl = (p * (1.0 - p))[:, None]
    e = g_zl[:, 0] * local("out", h7)[:, 0] + _act_err(zl) * p
    g_h7 = back("out", g_zl)
    g_y7 = g_h7 * _dsilu(y7)
    e += np.sum(np.abs(g_h7) * _act_err(y7) * np.abs(h7) + np.abs(g_y7) * local("p7", h6), axis=1)
    g_h6 = back("p7", g_y7)
    e += np.sum(np.abs(g_h6) * U32 * np.abs(h6), axis=1)
    g_h5 = g_h6
    g_y5 = g_h5 * _dsilu(y5)
    e += np.sum(np.abs(g_h5) * _act_err(y5) * np.abs(h5) + np.abs(g_y5) * local("r5", h4), axis=1)
    g_h4 = g_h6 + back("r5", g_y5)
    g_y4 = g_h4 * _dsilu(y4)
    e += np.sum(np.abs(g_h4) * _act_err(y4) * np.abs(h4) + np.abs(g_y4) * local("r4", h3), axis=1)
    g_h3 = back("r4", g_y4)
    nc = hc2.shape[1]
    for g_h2, y2, h2, n2, y1, h1, n1, x in ((g_h3[:, :nc], yc2, hc2, "c2", yc1, hc1, "c1", phi),
                                            (g_h3[:, nc:], ym2, hm2, "m2", ym1, hm1, "m1", feat)):
        g_y2 = g_h2 * _dsilu(y2)
        e += np.sum(np.abs(g_h2) * _act_err(y2) * np.abs(h2) + np.abs(g_y2) * local(n2, h1), axis=1)
        g_h1 = back(n2, g_y2)
        g_y1 = g_h1 * _dsilu(y1)
        e += np.sum(np.abs(g_h1) * _act_err(y1) * np.abs(h1) + np.abs(g_y1) * local(n1, x), axis=1)
        g_x = back(n1, g_y1)
        e += np.sum(np.abs(g_x) * 1.01 * U32 * np.abs(x), axis=1)
    return p, 2.0 * e


def quantile_linear(values, q):
    """Sec. 3.5: tau_coarse = quantile_q(P_coarse), read as linear interpolation between the
    order statistics v_(0) <= ... <= v_(m-1) at position h = q (m - 1):
    tau = v_(k) + (h - k) (v_(k+1) - v_(k)), k = floor(h) (v_(k+1) = v_(k) when k = m - 1)."""
    v = np.sort(np.asarray(values, dtype=np.float64).ravel())
    m = v.size
    if m == 0:
        raise ValueError("empty")
    h = float(q) * float(m - 1)
    k = int(math.floor(h))
    g = h - k
    v0 = v[k]
    v1 = v[k + 1] if k + 1 < m else v0
    return v0 + g * (v1 - v0)


def coarse_shape(grid, stride):
    """Sec. 3.5: the coarse grid takes every stride-th point in both directions, starting at the
    first; coarse point (I, J) is fine point (stride I, stride J) and owns the cell of fine rows
    stride I .. stride I + stride - 1 and columns likewise (cut at the grid's edge)."""
    return (grid.ny + stride - 1) // stride, (grid.nx + stride - 1) // stride


def _grid_z(grid, rows, cols):
    xs = grid.a + (grid.b - grid.a) * cols / (grid.nx - 1) if grid.nx > 1 else np.full(cols.shape, grid.a)
    ys = grid.c + (grid.d - grid.c) * rows / (grid.ny - 1) if grid.ny > 1 else np.full(rows.shape, grid.c)
    return xs + 1j * ys


def hierarchical_mask(grid, prob_at, tau, stride=4, q=0.8, dilate=5, coarse=None):
    """Sec. 3.5 (hierarchical prediction) and Sec. 4 (the predicted region R):

    1. p on the coarse points (stride in both directions) -> P_coarse;
    2. tau_coarse = quantile_q(P_coarse) (``quantile_linear``);
    3. every cell whose coarse value is >= tau_coarse has p evaluated at all its fine
       points; every other fine point gets probability 0;
    4. R = {z : p(z) >= tau}, expanded by a dilate x dilate square structuring element
       (morphological dilation; neighbours outside the grid do not exist).

    prob_at(flat_indices) -> probabilities at those grid points (row-major, row <-> y).
    coarse: optional precomputed P_coarse (shape coarse_shape), used instead of prob_at on the
    coarse points (to feed another implementation's coarse values through the same rule).
    Returns dict(coarse, tau_coarse, selected, prob, mask, evals)."""
    ny, nx = grid.ny, grid.nx
    cy, cx = coarse_shape(grid, stride)
    ci, cj = np.meshgrid(np.arange(cy), np.arange(cx), indexing="ij")
    cflat = (stride * ci * nx + stride * cj).ravel()
    if coarse is None:
        coarse = np.asarray(prob_at(cflat), dtype=np.float64).reshape(cy, cx)
    else:
        coarse = np.asarray(coarse, dtype=np.float64).reshape(cy, cx)
    tau_c = quantile_linear(coarse, q)
    selected = coarse >= tau_c
    prob = np.zeros((ny, nx))
    fine = []
    for I, J in zip(*np.nonzero(selected)):
        for i in range(stride * I, min(ny, stride * I + stride)):
            for j in range(stride * J, min(nx, stride * J + stride)):
                fine.append(i * nx + j)
    fine = np.array(fine, dtype=np.int64)
    if fine.size:
        prob.ravel()[fine] = np.asarray(prob_at(fine), dtype=np.float64)
    hit = prob >= tau
    r = (dilate - 1) // 2
    mask = np.zeros((ny, nx), dtype=np.uint8)
    for i, j in zip(*np.nonzero(hit)):
        mask[max(0, i - r):i + r + 1, max(0, j - r):j + r + 1] = 1
    return dict(coarse=coarse, tau_coarse=tau_c, selected=selected, prob=prob, mask=mask,
                evals=int(cflat.size + fine.size))


def mask_predict(params, gfeat, eig, grid, tau, stride=4, q=0.8, dilate=5):
    """Sec. 3.5 / Sec. 4 with the network of Sec. 3.2 as the probability (float64)."""
    nx = grid.nx

    def prob_at(flat):
        flat = np.asarray(flat, dtype=np.int64)
        z = _grid_z(grid, (flat // nx).astype(np.float64), (flat % nx).astype(np.float64))
        return mlp_prob(params, gfeat, eig, z)

    return hierarchical_mask(grid, prob_at, tau, stride=stride, q=q, dilate=dilate)


def mask_points_z(grid, flat):
    """Grid points z at flat row-major indices (Sec. 2.1 grid, inclusive end points)."""
    flat = np.asarray(flat, dtype=np.int64)
    return _grid_z(grid, (flat // grid.nx).astype(np.float64), (flat % grid.nx).astype(np.float64))


def dilate(binary, side):
    """Morphological dilation of a 2-D boolean map by a side x side square centred on each point
    (side odd; neighbours outside the map do not exist)."""
    b = np.asarray(binary, dtype=bool)
    r = (side - 1) // 2
    out = np.zeros_like(b)
    for i, j in zip(*np.nonzero(b)):
        out[max(0, i - r):i + r + 1, max(0, j - r):j + r + 1] = True
    return out


def calibrate_tau(prob, labels, taus, pred_dilate=5, label_dilate=3, median_min=0.90, p10_min=0.75):
    """Sec. 3.6, threshold calibration on a validation set of matrices (one probability map and
    one ground-truth label map per matrix, same grid):

    for each candidate tau (ascending): S_hat = {p >= tau} dilated by a pred_dilate square, the
    labels dilated by a label_dilate square, recall = |S_hat_dil & S_dil| / |S_dil| per matrix
    (1 when S_dil is empty); a candidate qualifies when median(recall) >= median_min and
    P10(recall) >= p10_min, both quantiles by ``quantile_linear`` (q = 0.5 and 0.1).  tau* is
    the smallest qualifying candidate, as the paper writes it; recall cannot rise with tau, so
    that is the first candidate whenever any qualifies.  The largest qualifying candidate (the
    one that predicts the fewest points within the same recall bounds) is returned too.

    Returns dict(recall [nval, ntau], median [ntau], p10 [ntau], index, index_max (-1 if no
    candidate qualifies))."""
    prob = np.asarray(prob, dtype=np.float64)
    labels = np.asarray(labels)
    nval = prob.shape[0]
    taus = np.asarray(taus, dtype=np.float64)
    recall = np.zeros((nval, len(taus)))
    for m in range(nval):
        lab = dilate(labels[m] != 0, label_dilate)
        nlab = int(lab.sum())
        for k, tau in enumerate(taus):
            if nlab == 0:
                recall[m, k] = 1.0
                continue
            hit = int((dilate(prob[m] >= tau, pred_dilate) & lab).sum())
            recall[m, k] = hit / nlab
    med = np.array([quantile_linear(recall[:, k], 0.5) for k in range(len(taus))])
    p10 = np.array([quantile_linear(recall[:, k], 0.1) for k in range(len(taus))])
    ok = np.flatnonzero((med >= median_min) & (p10 >= p10_min))
    return dict(recall=recall, median=med, p10=p10, index=int(ok[0]) if ok.size else -1,
                index_max=int(ok[-1]) if ok.size else -1)
