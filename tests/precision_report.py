"""Precision form report: the gripper scene at r = 64 stepped in the FP64 form and in
the mixed form (FP32 Hessian blocks, products and preconditioner) from the same
initial state.

Per step: Newton iterations and wall time of each form, the largest vertex distance
between the two trajectories, the relative difference of their incremental-potential
energies at the accepted states, and the FP64 gradient norm at each accepted state
(both forms stop when the Newton direction is below the same tolerance, so both norms
are small and comparable); at the end the GPU intersection count of the mixed state.

    python tests/precision_report.py --steps 10 --res 64 > report.md
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--res", type=int, default=64)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--newton-max", type=int, default=1000)
    args = ap.parse_args()
    import torch

    import scenegen as sg
    from paper_2311_05945_amd import zema
    sa = sg.gripper(args.seed, r=args.res, steps=args.steps)
    sb = sg.gripper(args.seed, r=args.res, steps=args.steps, precision=1)
    sa.params.newton_max = sb.params.newton_max = args.newton_max
    A = zema.Scene(sa)
    B = zema.Scene(sb)
    n3 = 3 * A.n_soft_verts
    print(f"# Precision form, gripper r={args.res} seed {args.seed}: {A.n_soft_verts} soft vertices, "
          f"{A.n_tets} tets, {A.n_tris} surface triangles\n")
    print("| step | Newton FP64 | Newton mixed | ms FP64 | ms mixed | max vertex distance (m) | "
          "energy rel. diff | |g| FP64 state | |g| mixed state |")
    print("|---|---|---|---|---|---|---|---|---|")
    ta = tb = 0.0
    na = nb = 0
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st_a = A.step(1)[0]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st_b = B.step(1)[0]
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ta += t1 - t0
        tb += t2 - t1
        na += st_a["newton_iters"]
        nb += st_b["newton_iters"]
        ya = A.get_state()[0]
        yb = B.get_state()[0]
        dx = (ya[:n3] - yb[:n3]).view(-1, 3).norm(dim=1).max().item()
        ea, ga = A.ip_assemble(ya, hess=False)
        eb, gb = A.ip_assemble(yb, hess=False)       # FP64 evaluation of the mixed state
        de = abs(eb[6] - ea[6]) / abs(ea[6])
        print(f"| {k + 1} | {st_a['newton_iters']} | {st_b['newton_iters']} | {1e3 * (t1 - t0):.0f} | "
              f"{1e3 * (t2 - t1):.0f} | {dx:.2e} | {de:.2e} | {ga.norm().item():.2e} | {gb.norm().item():.2e} |",
              flush=True)
    ni, nv, nu, _ = B.intersection_count(B.get_state()[0], cap=0)
    print(f"\nTotals: FP64 {na} Newton iterations in {ta:.2f} s, mixed {nb} in {tb:.2f} s "
          f"(speed-up {ta / tb:.2f}x); mixed final state: {ni} intersecting pairs, {nv} inverted tets, "
          f"{nu} uncertain.")


if __name__ == "__main__":
    main()
