"""Training and evaluation of the learned preconditioning stage (GPU, through the C ABI).

Pairs (residual, error) come from plain space-time multigrid: for a right-hand side b the
reference solution x* is an FGMRES solve to a 1e-11 relative residual, and the iterates
x_{k+1} = x_k + V(b - S x_k) (x_0 = 0, FP64 V-cycle) give r_k = b - S x_k and
e_k = x* - x_k.  The network is trained by the library's BF16 kernels with Adam on
L = ||C(r) - e||^2 / ||e||^2.  Because the network is a convolution on the node lattice,
weights trained on a small domain with the same mesh width, degrees and time step apply to
the full problem.

CLI:  python -m paper_2408_04372_amd.learned train --config 5 --solves 400 --out w.npy
      python -m paper_2408_04372_amd.learned gain --config 5 --weights w.npy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _imports():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import torch
    import stmg_inputs as si
    from paper_2408_04372_amd import Handle
    return torch, si, Handle


def training_config(idx: int, cells: int = 16):
    """Same mesh width, degrees, time step and coefficient law as configuration idx on a
    smaller box of `cells` cells per direction."""
    torch, si, Handle = _imports()
    cfg = si.paper_config(idx)
    h = cfg.h[0]
    return cfg.replace(n_cells=(cells,) * 3, hi=(cells * h,) * 3, name=cfg.name + f"_train{cells}")


def default_channels(n_t: int):
    return [n_t, 16, 16, n_t]


def make_pairs(h, cfg, seeds, iters=(0, 1, 2, 3), log=None):
    """(r_k, e_k) device tensors for every seed and every k in iters."""
    torch, si, Handle = _imports()
    dev = torch.device("cuda:0")
    pairs = []
    for j, sd in enumerate(seeds):
        if log and j % 100 == 0:
            log(f"pairs: solve {j}")
        b = torch.from_numpy(si.random_slab_vector(cfg, int(sd))).to(dev).reshape(-1).contiguous()
        xs = torch.zeros_like(b)
        h.solve(b, xs, raise_on_noconv=False)
        x = torch.zeros_like(b)
        z = torch.empty_like(b)
        for k in range(max(iters) + 1):
            e = xs - x                      # training target e_k (data preparation, not the method)
            r = torch.empty_like(b)
            h.mg_step(b, x, r, z)           # r_k = b - S x_k, x_{k+1} = x_k + V r_k (library kernels)
            if k in iters:
                pairs.append((r, e))
    torch.cuda.synchronize()
    return pairs


def train(h, pairs, epochs: int = 4, lr: float = 2e-3, log=None):
    losses = []
    rng = np.random.default_rng(0)
    for ep in range(epochs):
        order = rng.permutation(len(pairs))
        tot = 0.0
        for i in order:
            r, e = pairs[i]
            tot += h.cnn_train_step(r, e, lr)
        losses.append(tot / len(pairs))
        if log:
            log(f"epoch {ep}: mean loss {losses[-1]:.4f}")
    return losses


MODES = ((0, "fp64"), (1, "fp32_vcycle"), (2, "learned"))


def gain(cfg, verts, coef, theta, channels, seeds, **kw):
    """Iterations and time to rtol of plain FP64 STMG, FP32-V-cycle STMG and the learned stage
    (which wraps the FP32 V-cycle) on held-out seeds."""
    torch, si, Handle = _imports()
    dev = torch.device("cuda:0")
    out = {key: [] for _, key in MODES}
    h = Handle(cfg, verts, coef, vcycle_dtypes=3, precision=2, **kw)
    h.cnn_create(channels)
    h.cnn_set_params(theta)
    b0 = torch.from_numpy(si.random_slab_vector(cfg, int(seeds[0]))).to(dev).reshape(-1).contiguous()
    x = torch.zeros_like(b0)
    for prec, key in MODES:
        h.set_precision(prec)
        x.zero_()
        h.solve(b0, x, raise_on_noconv=False)       # warm-up (workspace allocation)
        for sd in seeds:
            b = torch.from_numpy(si.random_slab_vector(cfg, int(sd))).to(dev).reshape(-1).contiguous()
            x.zero_()
            inf = h.solve(b, x, raise_on_noconv=False)
            out[key].append(inf)
    h.close()
    summ = {}
    for key in out:
        its = [i["iterations"] for i in out[key]]
        ts = [i["seconds"] for i in out[key]]
        summ[key] = {"iterations_mean": float(np.mean(its)), "seconds_mean": float(np.mean(ts)),
                     "rel_residual_max": float(max(i["rel_residual"] for i in out[key])),
                     "cnn_used": int(sum(i["cnn_used"] for i in out[key])),
                     "cnn_fallbacks": int(sum(i["cnn_fallbacks"] for i in out[key]))}
    base = summ["fp32_vcycle"]
    summ["speedup_time_vs_fp32"] = base["seconds_mean"] / summ["learned"]["seconds_mean"]
    summ["iteration_ratio_vs_fp32"] = summ["learned"]["iterations_mean"] / base["iterations_mean"]
    return summ


def _log(msg):
    print(msg, flush=True)


def train_for_config(idx: int, solves: int, epochs: int, lr: float, cells: int = 16, log=_log, seed0: int = 1001):
    """Train a network for configuration idx on `solves` seeded right-hand sides."""
    torch, si, Handle = _imports()
    tcfg = training_config(idx, cells)
    verts, coef = si.draw_problem(tcfg)
    # plain FP64 multigrid for the reference solves and the stationary iterations
    h = Handle(tcfg, verts, coef, vcycle_dtypes=1, precision=0, omega=-1.0, rtol=1e-11, max_iter=300)
    ch = default_channels(tcfg.n_t)
    h.cnn_create(ch)
    rng = np.random.Generator(np.random.PCG64(7))
    parts = []
    for l in range(len(ch) - 1):
        parts.append(rng.standard_normal(27 * ch[l + 1] * ch[l]) * np.sqrt(2.0 / (27 * ch[l])) * 0.5)
        parts.append(np.zeros(ch[l + 1]))
    h.cnn_set_params(np.concatenate(parts).astype(np.float32))
    t0 = time.time()
    pairs = make_pairs(h, tcfg, range(seed0, seed0 + solves), log=log)
    log(f"{len(pairs)} pairs from {solves} solves on {tcfg.name} in {time.time() - t0:.1f} s")
    t0 = time.time()
    losses = train(h, pairs, epochs, lr, log=log)
    log(f"trained {epochs} epochs in {time.time() - t0:.1f} s")
    theta = h.cnn_get_params()
    h.close()
    return theta, ch, losses


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "gain"])
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--solves", type=int, default=400)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--cells", type=int, default=16)
    ap.add_argument("--weights", default=None)
    ap.add_argument("--out", default=None)
    ap.add_argument("--eval-cells", type=int, default=0, help="evaluate on this many cells per direction (0: full)")
    args = ap.parse_args()
    torch, si, Handle = _imports()
    if args.cmd == "train":
        theta, ch, losses = train_for_config(args.config, args.solves, args.epochs, args.lr, args.cells)
        if args.out:
            np.save(args.out, theta)
        print(json.dumps({"channels": ch, "losses": losses}))
    else:
        theta = np.load(args.weights)
        cfg = si.paper_config(args.config)
        if args.eval_cells:
            cfg = training_config(args.config, args.eval_cells)
        verts, coef = si.draw_problem(cfg)
        res = gain(cfg, verts, coef, theta, default_channels(cfg.n_t), seeds=range(3001, 3004), omega=-1.0,
                   rtol=1e-8, max_iter=300)
        print(json.dumps(res))


if __name__ == "__main__":
    main()
