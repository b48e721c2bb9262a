"""Training of the learned initial guess on trajectories the simulator generates.

Data: uneven grasp scenes (`scenegen.batch_scene`, seeds from 20000, disjoint from
the evaluation seeds from 10000) are stepped together as one batch with the explicit
initial guess; before every step the features of every soft vertex are recorded, after
it the step's target ((x^{t+1} - x^t) - h v^t) / s.  Training: Adam on the network's
own GPU kernels, mini-batches of 4096 vertex-steps drawn with a seeded generator.

    python -m paper_2311_05945_amd.warm_train --out weights.npy

The weights are written as a flat float32 array of 9603 parameters (W1, b1, ..., b4).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def collect(seeds, steps, newton_max=2000, device="cuda:0"):
    """Feature / target tensors (device, float32) of every soft vertex and step."""
    import torch

    import scenegen as sg
    from paper_2311_05945_amd import zema
    scenes = [sg.batch_scene(s, steps=steps) for s in seeds]
    for sc in scenes:
        sc.params.newton_max = newton_max
    B = zema.Scene.batch(scenes, device=device)
    log(f"data batch: {len(seeds)} scenes, {B.n_soft_verts} soft vertices, {B.n_tets} tets")
    feats, targs = [], []
    t0 = time.perf_counter()
    for k in range(steps):
        feats.append(B.features())
        st = B.step(1)
        targs.append(B.warm_target())
        it = [x["newton_iters"] for x in st]
        log(f"  step {k + 1}/{steps}: {time.perf_counter() - t0:.1f} s, newton max {max(it)} "
            f"(scene {it.index(max(it))}), mean {sum(it) / len(it):.1f}")
    return torch.cat(feats).contiguous(), torch.cat(targs).contiguous()


def train(X, T, iters, lr, seed, init_seed, device="cuda:0", batch=4096):
    import torch

    import scenegen as sg
    from paper_2311_05945_amd import zema
    M = zema.Mlp(sg.mlp_init(init_seed), device=device)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    hist = []
    t0 = time.perf_counter()
    for it in range(iters):
        idx = torch.randint(0, n, (batch,), generator=gen, dtype=torch.int64).to(torch.int32).to(device)
        rate = lr * (0.1 + 0.9 * 0.5 * (1.0 + np.cos(np.pi * it / iters)))   # cosine decay to lr / 10
        hist.append(M.train_step(X, T, idx, rate))
        if (it + 1) % 500 == 0:
            log(f"  iter {it + 1}/{iters}: loss {np.mean(hist[-500:]):.5f} ({time.perf_counter() - t0:.1f} s)")
    return M, hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--scenes", type=int, default=16)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--iters", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    seeds = list(range(20000, 20000 + args.scenes))
    X, T = collect(seeds, args.steps)
    log(f"{X.shape[0]} vertex-steps; target rms {float(T.pow(2).mean().sqrt()):.4f}")
    M, hist = train(X, T, args.iters, args.lr, args.seed, init_seed=args.seed + 1)
    np.save(args.out, M.get_weights())
    log(f"loss {hist[0]:.5f} -> {np.mean(hist[-100:]):.5f}; weights written to {args.out}")


if __name__ == "__main__":
    main()
