"""Training of the classifier of Sec. 3.2 on exact labels (Sec. 3.3, Sec. 3.4) and calibration
of its threshold (Sec. 3.6), on the GPU.

    python -m paper_2605_04550_amd.train_mask [--train 500] [--val 30] [--test 100] [--out FILE]

Data (all synthetic, the class of Sec. 3.3, eq. (matrix): n = 64, bandwidth beta ~ U{1..4},
entries U{-1, 0, 1}, A != A^T, cond(A) < 1e8): training matrices from seed base + 20000 + m,
validation matrices from base + 30000 + m, held-out test matrices from base + 6000 + m (the
label workload).  Labels: sigma_min(zI - A) <= 0.01 on the 100 x 100 grid over [-4, 4]^2, exact,
from the library's exclusion-region labelling (ps_label_batch).  Samples per matrix (Sec. 3.3,
balanced sampling): every sensitive point and max(10 n_pos, 200) seeded non-sensitive points.

Training (Sec. 3.4): binary cross-entropy, Adam with learning rate 1e-3, batch 512, at most 25
epochs, early stopping on the validation loss with patience 5 (the best epoch's weights kept).
The matrix-path inputs (f1 .. f30, g1 .. g3) are standardised by the training set's mean and
standard deviation; the standardisation is folded into the first matrix-path layer when the
weights are exported, so the exported parameter vector takes the raw features like any other.

Calibration (Sec. 3.6): the hierarchical predictor's probability maps of the validation
matrices and their exact labels through ps_mask_calibrate (5 x 5 dilation of the predictions,
3 x 3 of the labels, median recall >= 0.90 and 10th percentile >= 0.75, candidates 0.05 ..
0.94); tau* the smallest qualifying candidate.

Evaluation on the test matrices: recall of R (the prediction at tau*, dilated 5 x 5) against
the labels dilated 3 x 3 (as in the calibration), the fraction of the grid in R, and the
sensitive points outside R.

Output: a .npz with params (float32, the library's layout), tau, and the metrics; one JSON
line on stdout.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import api
from .features import band_features

# Layer shapes (out, in) of Sec. 3.2 in the order of the parameter vector (include/ps.h):
# c1, c2 (coordinate path), m1, m2 (matrix path), r4, r5 (residual block), p7, out.
LAYERS = (("c1", 64, 26), ("c2", 64, 64), ("m1", 128, 33), ("m2", 64, 128), ("r4", 128, 128), ("r5", 128, 128),
          ("p7", 64, 128), ("out", 1, 64))
NPARAM = sum(o * i + o for _, o, i in LAYERS)
GRID = (-4.0, 4.0, -4.0, 4.0, 100, 100)
EPS_LABEL = 0.01


class MaskMLP(torch.nn.Module):
    """The dual-path network of Sec. 3.2 as torch layers (float32), for training."""

    def __init__(self):
        super().__init__()
        self.lin = torch.nn.ModuleDict({name: torch.nn.Linear(i, o) for name, o, i in LAYERS})

    @staticmethod
    def fourier(x, y):
        """phi(c): [x, y], then sin, cos of 2^k x and 2^k y for k = 1 .. 6 (26 values)."""
        cols = [x, y]
        for k in range(1, 7):
            f = float(2 ** k)
            cols += [torch.sin(f * x), torch.sin(f * y), torch.cos(f * x), torch.cos(f * y)]
        return torch.stack(cols, dim=1)

    def forward(self, phi, feat):
        act = torch.nn.functional.silu
        hc = act(self.lin["c2"](act(self.lin["c1"](phi))))
        hm = act(self.lin["m2"](act(self.lin["m1"](feat))))
        h4 = act(self.lin["r4"](torch.cat([hc, hm], dim=1)))
        h6 = h4 + act(self.lin["r5"](h4))
        return self.lin["out"](act(self.lin["p7"](h6)))[:, 0]      # the logit

    def export(self, mu=None, sd=None):
        """The flat parameter vector (float32), with x -> (x - mu) / sd folded into m1."""
        parts = []
        for name, o, i in LAYERS:
            W = self.lin[name].weight.detach().double().cpu().numpy()
            b = self.lin[name].bias.detach().double().cpu().numpy()
            if name == "m1" and mu is not None:
                b = b - W @ (mu / sd)
                W = W / sd[None, :]
            parts += [W.ravel(), b]
        return np.concatenate(parts).astype(np.float32)

    def load_flat(self, params):
        p = np.asarray(params, dtype=np.float32).ravel()
        at = 0
        with torch.no_grad():
            for name, o, i in LAYERS:
                self.lin[name].weight.copy_(torch.from_numpy(p[at:at + o * i].reshape(o, i)))
                at += o * i
                self.lin[name].bias.copy_(torch.from_numpy(p[at:at + o]))
                at += o


def point_features(z, eig):
    """g1, g2, g3 of Sec. 3.1 eq. (dist) (lambda* the eigenvalue centroid)."""
    d = np.abs(z[:, None] - eig[None, :])
    return np.stack([d.min(axis=1), np.abs(z - eig.mean()), d.mean(axis=1)], axis=1)


def grid_z():
    a, b, c, d, nx, ny = GRID
    xs = np.array([a + (b - a) * j / (nx - 1) for j in range(nx)])
    ys = np.array([c + (d - c) * i / (ny - 1) for i in range(ny)])
    return (xs[None, :] + 1j * ys[:, None]).ravel()


def make_set(seeds, dev, feat_seed):
    """Matrices, their features and spectra, and exact labels on the grid."""
    import workloads as W
    mats = [W.paper_training_matrix(s) for s in seeds]
    feats, eigs = zip(*[band_features(b, feat_seed + k) for k, b in enumerate(mats)])
    handles = [api.BandedMatrix.from_band(b) for b in mats]
    grid = W.Grid(*GRID)
    batch = api.BandedBatch(handles, [grid] * len(mats))
    lab = batch.label(EPS_LABEL)
    labels = lab["label"].reshape(len(mats), GRID[5], GRID[4]).cpu().numpy()
    return dict(mats=mats, feats=np.array(feats), eigs=list(eigs), labels=labels, grid=grid)


def balanced_samples(s, rng):
    """(matrix index, flat point) of every sensitive point and max(10 n_pos, 200) others."""
    rows = []
    for m, lab in enumerate(s["labels"]):
        flat = lab.ravel()
        pos = np.flatnonzero(flat == 1)
        neg = np.flatnonzero(flat == 0)
        k = min(len(neg), max(10 * len(pos), 200))
        pick = np.concatenate([pos, rng.choice(neg, size=k, replace=False)])
        rows.append(np.stack([np.full(len(pick), m), pick], axis=1))
    return np.concatenate(rows)


def tensors(s, samples, z, dev):
    m, p = samples[:, 0], samples[:, 1]
    zz = z[p]
    g = np.empty((len(samples), 3))
    for k in np.unique(m):
        sel = m == k
        g[sel] = point_features(zz[sel], s["eigs"][k])
    feat = np.concatenate([s["feats"][m], g], axis=1)
    y = s["labels"].reshape(len(s["mats"]), -1)[m, p].astype(np.float32)
    return (torch.tensor(zz.real, dtype=torch.float32, device=dev), torch.tensor(zz.imag, dtype=torch.float32, device=dev),
            torch.tensor(feat, dtype=torch.float64, device=dev), torch.tensor(y, device=dev))


def dilate(binary, side):
    import scipy.ndimage as nd
    return nd.binary_dilation(binary, structure=np.ones((side, side), dtype=bool))


def main(argv=None):
    import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=500)
    ap.add_argument("--val", type=int, default=30)
    ap.add_argument("--test", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=25)
    ap.add_argument("--patience", type=int, default=5)
    ap.add_argument("--out", default="mask_net.npz")
    args = ap.parse_args(argv)
    dev = torch.device("cuda")
    torch.manual_seed(2605)
    rng = np.random.default_rng(W.SEED_BASE + 50)
    t0 = time.time()
    tr = make_set([W.SEED_BASE + 20000 + m for m in range(args.train)], dev, 1_000_000)
    va = make_set([W.SEED_BASE + 30000 + m for m in range(args.val)], dev, 2_000_000)
    te = make_set([W.SEED_BASE + 6000 + m for m in range(args.test)], dev, 3_000_000)
    print("train_mask: data (%d / %d / %d matrices) in %.1f s" % (args.train, args.val, args.test, time.time() - t0),
          file=sys.stderr, flush=True)
    z = grid_z()
    s_tr = balanced_samples(tr, rng)
    s_va = balanced_samples(va, rng)
    xtr, ytr_, ftr, ytr = tensors(tr, s_tr, z, dev)
    xva, yva_, fva, yva = tensors(va, s_va, z, dev)
    mu = ftr.mean(dim=0)
    sd = ftr.std(dim=0).clamp_min(1e-6)
    ftr_n = ((ftr - mu) / sd).float()
    fva_n = ((fva - mu) / sd).float()
    phi_tr = MaskMLP.fourier(xtr, ytr_)
    phi_va = MaskMLP.fourier(xva, yva_)
    net = MaskMLP().to(dev)
    opt = torch.optim.Adam(net.parameters(), lr=1e-3)
    lossf = torch.nn.BCEWithLogitsLoss()
    best, best_state, wait, history = math.inf, None, 0, []
    ntr = len(ytr)
    for ep in range(args.epochs):
        net.train()
        perm = torch.randperm(ntr, device=dev)
        tot = 0.0
        for i in range(0, ntr, 512):
            idx = perm[i:i + 512]
            opt.zero_grad()
            loss = lossf(net(phi_tr[idx], ftr_n[idx]), ytr[idx])
            loss.backward()
            opt.step()
            tot += float(loss.detach()) * len(idx)
        net.eval()
        with torch.no_grad():
            vl = float(lossf(net(phi_va, fva_n), yva))
        history.append((tot / ntr, vl))
        print("train_mask: epoch %d train loss %.4f validation loss %.4f" % (ep + 1, tot / ntr, vl),
              file=sys.stderr, flush=True)
        if vl < best:
            best, wait = vl, 0
            best_state = {k: v.detach().clone() for k, v in net.state_dict().items()}
        else:
            wait += 1
            if wait >= args.patience:
                break
    net.load_state_dict(best_state)
    params = net.export(mu.cpu().numpy(), sd.cpu().numpy())
    mnet = api.MaskNet(params)

    def maps(s):
        eig_t = [torch.tensor(e, dtype=torch.complex128, device=dev) for e in s["eigs"]]
        return mnet.predict_batch(s["grid"], s["feats"], eig_t, tau=0.05)

    pv = maps(va)
    cal = api.calibrate_tau(va["grid"], pv["prob"], torch.tensor(va["labels"], device=dev))
    if cal["index"] < 0:
        tau = cal["taus"][0]
        print("train_mask: no candidate meets the recall bounds; using %.2f" % tau, file=sys.stderr, flush=True)
    else:
        tau = cal["taus"][cal["index"]]
    # held-out test matrices: the hierarchical predictor at tau*
    eig_t = [torch.tensor(e, dtype=torch.complex128, device=dev) for e in te["eigs"]]
    pt = mnet.predict_batch(te["grid"], te["feats"], eig_t, tau=tau)
    masks = pt["mask"].cpu().numpy().astype(bool)
    rec, cov, missed = [], [], 0
    for m in range(len(te["mats"])):
        lab = te["labels"][m].astype(bool)
        dl = dilate(lab, 3)
        dp = masks[m]                     # R = {p >= tau*} dilated 5 x 5, as in the calibration
        rec.append(1.0 if dl.sum() == 0 else float((dl & dp).sum()) / float(dl.sum()))
        cov.append(float(masks[m].mean()))
        missed += int((lab & ~masks[m]).sum())
    rec = np.array(rec)
    out = dict(params=params, tau=np.float64(tau), history=np.array(history),
               cal_median=cal["median"].cpu().numpy(), cal_p10=cal["p10"].cpu().numpy(),
               test_recall=rec, test_coverage=np.array(cov))
    np.savez_compressed(args.out, **out)
    line = dict(samples_train=int(ntr), samples_val=int(len(yva)), epochs=len(history),
                best_val_loss=best, tau_star=tau, cal_median=float(cal["median"][max(cal["index"], 0)]),
                cal_p10=float(cal["p10"][max(cal["index"], 0)]),
                test_matrices=len(te["mats"]), test_recall_median=float(np.median(rec)),
                test_recall_p10=float(np.percentile(rec, 10)), test_coverage_mean=float(np.mean(cov)),
                test_sensitive_points=int(te["labels"].sum()), test_sensitive_outside_R=missed,
                seconds=time.time() - t0, out=args.out)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
