"""Training driver of the learned spectral-interval predictor.

The network (9-64-64-64-3, tanh, FP32) is trained on the GPU by the library's
own kernels (adl_mlp_forward / adl_mlp_mse_grad / adl_mlp_backward /
adl_mlp_adam_step).  Training data come from the method itself: for each
seeded random coefficient field the library computes the field statistics
(adl_field_stats), the power-iteration spectral radius (adl_spectral_bound)
and the phi_1 Leja degree and substeps at that interval (adl_leja_phi); the
dimensionless inputs and targets are formed by adl_learned_features /
adl_learned_targets.  PyTorch only provides device buffers.

    python -m paper_2307_12276_amd.learned --samples 10000 --out <weights file>
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "learned_bound_weights.f32")
META = os.path.join(HERE, "learned_bound_meta.json")

POWER_MAX_ITER = 2000
POWER_RTOL = 1e-7
LABEL_TOL = 1e-8
LABEL_SAFETY = 1.1


def _sample(seed):
    sys.path.insert(0, os.path.dirname(HERE))
    import workloads as W
    return W.learned_sample(seed)


def label_sample(d, A, torch):
    """Features and labels of one sample (all arithmetic in the library)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    op = A.Op(t(d["Dxx"]), t(d["Dxy"]), t(d["Dyy"]), d["hx"], d["hy"], d["bc"], A.STORAGE_FP64,
              ax_c=d["ax_c"], ay_c=d["ay_c"])
    feats = torch.empty(9, dtype=torch.float32, device=dev)
    op.field_stats(d["dt"], feats)
    ag, _ = op.spectral_bound(A.BOUND_GERSHGORIN)
    alpha, its = op.spectral_bound(A.BOUND_POWER, max_iter=POWER_MAX_ITER, rtol=POWER_RTOL, seed=1)
    lam = op.last_power_estimate()
    v = t(np.random.default_rng(0).standard_normal((d["ny"], d["nx"])))
    out = torch.empty_like(v)
    st = op.leja_phi(1, d["dt"], v, out, LABEL_TOL)
    f = feats.cpu().tolist()
    x = A.learned_features(f, -ag)
    y = A.learned_targets(f, -ag, lam, st["max_degree"], max(st["substeps"], 1))
    op.close()
    return f, x, y, {"power_iters": its, "rho": lam, "degree": st["max_degree"], "substeps": st["substeps"]}


def make_dataset(n, seed0=0, workers=8, log=print):
    import torch
    import paper_2307_12276_amd as A
    F, X, Y, info = [], [], [], []
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for i, d in enumerate(ex.map(_sample, range(seed0, seed0 + n), chunksize=8)):
            f, x, y, meta = label_sample(d, A, torch)
            F.append(f)
            X.append(x)
            Y.append(y)
            info.append(meta)
            if (i + 1) % 500 == 0:
                log("labelled %d/%d samples (%.0f s)" % (i + 1, n, time.time() - t0))
    return np.array(F, np.float32), np.array(X, np.float32), np.array(Y, np.float32), info


def init_weights(seed=0):
    """Glorot-uniform weights, zero biases, packed W_l [in][out] then b_l."""
    rng = np.random.default_rng(seed)
    sizes = (9, 64, 64, 64, 3)
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = math.sqrt(6.0 / (a + b))
        parts.append(rng.uniform(-lim, lim, size=a * b))
        parts.append(np.zeros(b))
    return np.concatenate(parts).astype(np.float32)


def train(X, Y, epochs=300, batch=256, lr=2e-3, seed=0, log=print):
    """Adam on the MSE of the dimensionless targets; returns (W on host, history)."""
    import torch
    import paper_2307_12276_amd as A
    dev = torch.device("cuda", torch.cuda.current_device())
    n = X.shape[0]
    Xd = torch.from_numpy(X).to(dev)
    Yd = torch.from_numpy(Y).to(dev)
    W = torch.from_numpy(init_weights(seed)).to(dev)
    m1 = torch.zeros_like(W)
    m2 = torch.zeros_like(W)
    dW = torch.zeros_like(W)
    cache = torch.empty((batch, A.MLP_CACHE_PER_ROW), dtype=torch.float32, device=dev)
    Yp = torch.empty((batch, 3), dtype=torch.float32, device=dev)
    dY = torch.empty_like(Yp)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(seed)
    hist = []
    step = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(dev)
        tot = 0.0
        nb = 0
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            xb = Xd.index_select(0, idx).contiguous()
            yb = Yd.index_select(0, idx).contiguous()
            A.mlp_forward(W, xb, Yp, cache)
            A.mlp_mse_grad(Yp, yb, dY, loss)
            A.mlp_backward(W, cache, dY, dW)
            step += 1
            lr_t = lr * (0.5 * (1 + math.cos(math.pi * ep / epochs)) * 0.9 + 0.1)
            A.mlp_adam_step(W, dW, m1, m2, step, lr_t)
            tot += float(loss.item()) if (s // batch) % 16 == 0 else 0.0
            nb += 1 if (s // batch) % 16 == 0 else 0
        hist.append(tot / max(nb, 1))
        if (ep + 1) % 50 == 0:
            log("epoch %d loss %.5f" % (ep + 1, hist[-1]))
    return W.cpu().numpy(), hist


def predict(W, X):
    import torch
    import paper_2307_12276_amd as A
    dev = torch.device("cuda", torch.cuda.current_device())
    Wd = torch.from_numpy(np.ascontiguousarray(W, np.float32)).to(dev)
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(dev)
    Y = torch.empty((X.shape[0], 3), dtype=torch.float32, device=dev)
    A.mlp_forward(Wd, Xd, Y)
    return Y.cpu().numpy()


def save(W, meta, path=WEIGHTS, meta_path=META):
    np.asarray(W, np.float32).tofile(path)
    with open(meta_path, "w") as fh:
        json.dump(meta, fh, indent=1)


def load(path=WEIGHTS):
    W = np.fromfile(path, dtype=np.float32)
    if W.size != 9155:
        raise ValueError("bad weight file %s" % path)
    return W


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=10000)
    ap.add_argument("--holdout", type=float, default=0.1)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--dataset-out", default=None)
    args = ap.parse_args()
    log = lambda *a: print(*a, flush=True)
    t0 = time.time()
    F, X, Y, info = make_dataset(args.samples, workers=args.workers, log=log)
    t_label = time.time() - t0
    if args.dataset_out:
        np.savez(args.dataset_out, F=F, X=X, Y=Y)
    n_hold = int(args.holdout * len(X))
    Xtr, Ytr, Xte, Yte = X[n_hold:], Y[n_hold:], X[:n_hold], Y[:n_hold]
    t0 = time.time()
    W, hist = train(Xtr, Ytr, epochs=args.epochs, log=log)
    t_train = time.time() - t0
    P = predict(W, Xte)
    rho_rel = np.abs(10.0 ** ((P[:, 0] - Yte[:, 0]) / 10.0) - 1.0)
    deg_rel = np.abs(P[:, 1] / Yte[:, 1] - 1.0)
    meta = {"samples": int(len(X)), "holdout": int(n_hold), "epochs": args.epochs,
            "label_seconds": t_label, "train_seconds": t_train, "final_loss": hist[-1],
            "holdout_rho_rel_err_median": float(np.median(rho_rel)),
            "holdout_rho_rel_err_p95": float(np.percentile(rho_rel, 95)),
            "holdout_rho_rel_err_max": float(np.max(rho_rel)),
            "holdout_degree_rel_err_median": float(np.median(deg_rel)),
            "holdout_degree_rel_err_p95": float(np.percentile(deg_rel, 95)),
            "power_iters_mean": float(np.mean([m["power_iters"] for m in info])),
            "power_iteration": {"max_iter": POWER_MAX_ITER, "rtol": POWER_RTOL},
            "label_tol": LABEL_TOL}
    save(W, meta, args.out, os.path.splitext(args.out)[0].replace("_weights", "_meta") + ".json"
         if args.out != WEIGHTS else META)
    log(json.dumps(meta))


if __name__ == "__main__":
    main()
