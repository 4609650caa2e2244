"""Training of the local-basis surrogate network on the GPU.

Pairs (input features of a subdomain -> its exact local basis, the
solutions of the basis problems of Section 2.1) come from the library's
own local solver: FP64 contexts on synthetic log-normal fields, their
interior subdomains exported with rmrcm_export_local.  Training runs on
the network's own HIP kernels (rmrcm_cnn_train_step: forward, backward,
Adam); this module only draws fields, stacks the pairs in device memory
and schedules mini-batches.

    python -m paper_2009_07965_amd.learned --pairs 200000 --out cnn16.bin
"""

from __future__ import annotations

import argparse
import json
import time

import numpy as np

from .rmrcm import Net, Solver, rmrcm_export_local


def init_params(S, C, L, R, seed=0):
    """He-normal convolution weights, zero biases and mean field."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(L):
        co = R if l == L - 1 else C
        ci = 2 if l == 0 else C
        std = np.sqrt(2.0 / (ci * 9)) * (0.1 if l == L - 1 else 1.0)
        parts.append(rng.standard_normal(co * ci * 9) * std)
        parts.append(np.zeros(co))
    parts.append(np.zeros(R * S * S))
    return np.concatenate(parts).astype(np.float32)


def generate_pairs(n_pairs, sub=16, seg=4, m=16, seed=4000, log_var=(2.0, 5.0), lam=(0.02, 0.2),
                   device="cuda:0", verbose=False):
    """(x [N,2,S,S] float32, t [N,R,S,S] float32) on the device, from the
    interior subdomains of FP64 setups on random log-normal fields
    (m x m subdomains of sub^2 cells, segments of seg cells, alpha 1)."""
    import torch
    from workloads.fields import lognormal_grf
    from workloads.problems import dirichlet_we
    R = 4 * (sub // seg)
    n = sub * m
    rng = np.random.default_rng(seed)
    xs, ts, got, f = [], [], 0, 0
    dev = torch.device(device)
    while got < n_pairs:
        lv = float(rng.uniform(*log_var))
        lm = float(rng.uniform(*lam))
        K = lognormal_grf(n, n, lm, lv, seed=seed * 100000 + f)
        bct, _bcv = dirichlet_we(n, n)
        S = Solver(n, n, K, bct, sub, sub, seg)
        try:
            feats = torch.zeros((m * m, 2, sub, sub), dtype=torch.float32, device=dev)
            basis = torch.zeros((m * m, R, sub * sub), dtype=torch.float64, device=dev)
            interior = rmrcm_export_local(S.ctx, feats, basis)
        finally:
            S.close()
        idx = torch.from_numpy(np.nonzero(interior)[0]).to(dev)
        xs.append(feats.index_select(0, idx))
        ts.append(basis.index_select(0, idx).float().reshape(-1, R, sub, sub))
        got += int(idx.numel())
        f += 1
        if verbose and f % 100 == 0:
            print("  fields %d, pairs %d" % (f, got), flush=True)
    x = torch.cat(xs)[:n_pairs].contiguous()
    t = torch.cat(ts)[:n_pairs].contiguous()
    return x, t


def predict(net, x, batch=None):
    import torch
    batch = batch or net.max_batch
    y = torch.empty((x.shape[0], net.R, net.S, net.S), dtype=torch.float32, device=x.device)
    for k in range(0, x.shape[0], batch):
        net.forward(x[k:k + batch], y[k:k + batch])
    torch.cuda.synchronize()
    return y


def rel_error(y, t):
    """Mean over samples of ||y - t|| / ||t|| (all basis fields of a patch)."""
    d = (y - t).reshape(y.shape[0], -1).double().norm(dim=1)
    n = t.reshape(t.shape[0], -1).double().norm(dim=1)
    return float((d / n).mean())


def train(net, x, t, epochs=10, batch=256, lr=1e-3, seed=0, x_val=None, t_val=None, log=None):
    """Mini-batch Adam over shuffled pairs; returns the per-epoch history."""
    import torch
    rng = np.random.default_rng(seed)
    N = x.shape[0]
    hist = []
    for ep in range(epochs):
        t0 = time.perf_counter()
        perm = torch.from_numpy(rng.permutation(N)).to(x.device)
        losses = []
        lr_ep = lr * (0.5 ** (ep // max(1, epochs // 3)))
        for k in range(0, N - batch + 1, batch):
            idx = perm[k:k + batch]
            xb = x.index_select(0, idx).contiguous()
            tb = t.index_select(0, idx).contiguous()
            want = (k // batch) % 50 == 0
            l = net.train_step(xb, tb, lr_ep, want_loss=want)
            if want:
                losses.append(l)
        torch.cuda.synchronize()
        rec = {"epoch": ep, "lr": lr_ep, "loss": float(np.mean(losses)) if losses else None,
               "seconds": time.perf_counter() - t0}
        if x_val is not None:
            rec["val_rel_error"] = rel_error(predict(net, x_val), t_val)
        hist.append(rec)
        if log:
            log(rec)
    return hist


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=200000)
    ap.add_argument("--val", type=int, default=4096)
    ap.add_argument("--sub", type=int, default=16)
    ap.add_argument("--seg", type=int, default=4)
    ap.add_argument("--width", type=int, default=32)
    ap.add_argument("--layers", type=int, default=6)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default="cnn.bin")
    args = ap.parse_args()
    R = 4 * (args.sub // args.seg)
    t0 = time.perf_counter()
    x, t = generate_pairs(args.pairs, args.sub, args.seg, seed=4000, verbose=True)
    xv, tv = generate_pairs(args.val, args.sub, args.seg, seed=9000)
    t_gen = time.perf_counter() - t0
    net = Net(args.sub, args.width, args.layers, R, max_batch=256)
    net.set_params(init_params(args.sub, args.width, args.layers, R, seed=1))
    base = rel_error(predict(net, xv), tv)
    hist = train(net, x, t, args.epochs, 256, args.lr, 0, xv, tv,
                 log=lambda r: print(json.dumps(r), flush=True))
    net.save(args.out)
    print(json.dumps({"pairs": args.pairs, "generate_s": t_gen, "untrained_val_rel_error": base,
                      "final": hist[-1], "params": net.num_params}), flush=True)
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
