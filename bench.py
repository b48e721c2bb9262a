#!/usr/bin/env python
"""Benchmark of the plain FP64 Newton step on one MI355X.

Workload: the gripper scene -- a soft ellipsoid (semi-axes from the seed, voxelised
on an r^3 grid, E = 5e4 Pa, nu = 0.45) squeezed by two driven affine finger boxes
closing at 0.05 m/s, gravity, dt = 0.005 s, mu = 0.8, d-hat = 1e-3 m, Newton tolerance
1e-6 * dt, `--steps` time steps from rest.  Inputs are generated on the host and
copied to HBM before the timed region; the timed region is the K Newton time steps.

Prints one JSON line with the throughput (sim steps/s), Newton iterations per step,
the roofline figure of the dominant kernel (the PCG iteration: block-sparse product,
vector update and inner products in one launch; HIP events on the library's stream
around every replayed chunk of 16 iterations during a short pass of the next steps,
which checks convergence after every chunk and so is kept out of the throughput
figure), the
batched / learned / mixed-precision forms against the plain form on a sample of
uneven grasp scenes, and the CPU oracle timed on a bounded sample of the same
workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sim steps/s + Newton iters/step, learned+batched vs plain at same tol, 1 GPU"
HBM_PEAK_GBS = 8000.0
GROUPS_T = {"spmv": 0, "tet": 1, "contact": 2, "query": 3, "ccd": 4}
GROUPS = 4  # batch objects (and streams) of the batched forms: the device's hardware queues


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(scene, seconds, max_steps=20):
    """The oracle as it stands, timed on the host cores: the first steps of the same
    trajectory until `seconds` of CPU time have been spent (at least one step)."""
    from oracle import ref
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    used = ref.set_threads(threads)
    R = ref.RefScene(scene)
    t = 0.0
    n = 0
    newton = 0
    while n < max_steps and (n == 0 or t < seconds):
        t0 = time.perf_counter()
        st = R.step(1)[0]
        t += time.perf_counter() - t0
        n += 1
        newton += st["newton_iters"]
        log(f"cpu oracle step {n}: {t:.1f} s total, newton {st['newton_iters']}, pcg {st['pcg_iters']}")
    return {"value": n / t, "unit": "sim steps/s", "cores": used, "kind": "oracle",
            "sample": f"first {n} steps of the same trajectory ({newton} Newton iterations, {t:.1f} s; "
                      f"these early steps include the contact-free approach of the fingers)"}


def hbm_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter profile, or None when
    the profile is missing or the kernel's source changed since it was taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "pcg_iteration_gripper_r32_hbm_counters.md")
    src = os.path.join(ROOT, "paper_2311_05945_amd", "csrc", "k_sparse.hip")
    if not os.path.exists(prof):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for line in open(prof):
        f = line.split()
        if len(f) == 6 and f[0] == "traffic" and f[1] == kernel and f[5] == sha:
            return float(f[3])
    return None


def run_form(zema, scenes, steps, batched, learned=None, mixed=False, chunk=5):
    """Steps every scene `steps` times; returns (wall seconds, stats list, intersections)."""
    import torch
    for sc in scenes:
        sc.params.precision = 1 if mixed else 0
        sc.params.warm_start = 1 if learned is not None else 0
    # batched: the scenes in GROUPS batch objects on as many streams, stepped together
    # (zema_step_group); each batch takes all its steps in one call, every scene
    # starting its next step as soon as it has converged
    objs = zema.batch_group(scenes, GROUPS)[0] if batched else [zema.Scene(sc) for sc in scenes]
    for o in objs:
        if learned is not None:
            o.set_mlp(learned)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    if batched:
        for st in zema.step_group(objs, steps):
            stats += st
    for o in objs if not batched else []:
        done = 0
        while done < steps:
            n = min(chunk, steps - done)
            stats += o.step(n)
            done += n
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    inter = 0
    for o in objs:
        ni, nv, nu, _ = o.intersection_count(o.get_state()[0], cap=0)
        inter += ni + nv + nu
    return t, stats, inter


def forms(args, zema):
    """The batched, learned and mixed-precision forms against the plain form, on a
    sample of uneven grasp scenes at the same Newton tolerance."""
    import numpy as np

    import scenegen as sg
    seeds = list(range(args.form_seed, args.form_seed + args.form_scenes))
    mk = lambda: [sg.batch_scene(s, steps=args.form_steps) for s in seeds]
    mlp = None
    if os.path.exists(args.mlp):
        mlp = zema.Mlp(np.load(args.mlp))
    out = {"sample": f"{len(seeds)} uneven grasp scenes (seeds {seeds[0]}-{seeds[-1]}), {args.form_steps} steps "
                     f"each from rest, dt=0.005 s, Newton tol 1e-6 dt",
           "network": os.path.basename(args.mlp) if mlp is not None else None,
           "batched_as": f"{GROUPS} batch objects of similar size on {GROUPS} HIP streams, stepped together "
                         f"(zema_step_group); plain: one scene object after the other"}
    cases = [("plain", False, None, False), ("batched", True, None, False)]
    if mlp is not None:
        cases += [("learned", False, mlp, False), ("batched_learned", True, mlp, False),
                  ("batched_learned_mixed", True, mlp, True)]
    total = len(seeds) * args.form_steps
    # untimed warm-up of the grouped batch path (streams, host threads, first launches)
    run_form(zema, mk(), 2, True)
    for name, batched, learned, mixed in cases:
        t, st, inter = run_form(zema, mk(), args.form_steps, batched, learned, mixed)
        newton = sum(x["newton_iters"] for x in st)
        out[name] = {"steps_per_s": total / t, "newton_iters_per_step": newton / total,
                     "wall_s": t, "intersections": inter,
                     "learned_start_kept": (sum(x["warm_learned"] for x in st) / total) if learned else None}
        log(f"form {name}: {total / t:.2f} scene-steps/s, newton/step {newton / total:.2f}, "
            f"intersections {inter}")
    base = out["plain"]["steps_per_s"]
    for name, *_ in cases[1:]:
        out[name]["speedup_vs_plain"] = out[name]["steps_per_s"] / base
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--res", type=int, default=32)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--timer", default="spmv", choices=sorted(GROUPS_T))
    ap.add_argument("--chunk", type=int, default=10, help="steps per library call (progress lines)")
    ap.add_argument("--timing-steps", type=int, default=5, help="steps of the roofline pass after the timed run")
    ap.add_argument("--no-forms", action="store_true", help="skip the batched / learned / mixed comparison")
    ap.add_argument("--autotune", action="store_true", help="pick the PCG launch shapes by timing (default: fixed)")
    ap.add_argument("--no-graph", action="store_true", help="launch PCG kernels individually")
    ap.add_argument("--copy-probe", action="store_true", help="run a 256 MiB device copy (counter scaling)")
    ap.add_argument("--form-scenes", type=int, default=32)
    ap.add_argument("--form-steps", type=int, default=16)
    ap.add_argument("--form-seed", type=int, default=10000)
    ap.add_argument("--mlp", default=os.path.join(ROOT, "paper_2311_05945_amd", "warm_mlp.npy"))
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import scenegen as sg
    from paper_2311_05945_amd import zema

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    sc = sg.gripper(args.seed, r=args.res, steps=args.steps)
    tuned = None
    if args.warmup > 0:
        W = zema.Scene(sc)
        W.step(args.warmup)
        if args.autotune:
            lanes, ub, us = W.autotune()
            tuned = {"spmv_lanes": lanes, "update_block": ub, "us_per_pcg_iter": us}
            log(f"autotuned PCG shapes: {lanes} lanes per soft row, update block {ub}, {us:.2f} us/iteration")
        del W
    G = zema.Scene(sc)
    if args.no_graph:
        G.tune(zema.TUNE_PCG_GRAPH, 0)
    if tuned is not None:
        G.tune(zema.TUNE_SPMV_LANES, tuned["spmv_lanes"])
        G.tune(zema.TUNE_UPDATE_BLOCK, tuned["update_block"])
    log(f"scene: {G.n_soft_verts} soft vertices, {G.n_tets} tets, {G.n_dof} DOFs, {G.n_tris} surface triangles")
    group = GROUPS_T[args.timer]
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < args.steps:
        n = min(args.chunk, args.steps - done)
        stats += G.step(n)
        done += n
        log(f"steps {done}/{args.steps}: {time.perf_counter() - t0:.2f} s, newton/step "
            f"{sum(s['newton_iters'] for s in stats) / len(stats):.2f}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    # roofline pass: the next steps of the same trajectory with HIP events around the
    # timed kernel (PCG: every replayed chunk of 16 iterations; timed solves check
    # convergence after every chunk, so this pass is not part of the throughput figure)
    G.kernel_timer(group, True)
    torch.cuda.synchronize()
    tr0 = time.perf_counter()
    rstats = G.step(args.timing_steps)
    torch.cuda.synchronize()
    t_roof = time.perf_counter() - tr0
    ms_k, launches, bytes_k = G.kernel_time(group)
    log(f"roofline pass: {args.timing_steps} steps, {launches} launches of {args.timer}, {ms_k:.1f} ms")
    traffic = None
    kname = {"spmv": f"pcg_cg_kernel<double,{G.spmv_lanes()},false>"}.get(args.timer, args.timer)
    if args.timer == "spmv" and not G.params.precision:
        traffic = hbm_traffic(kname)
    newton = sum(s["newton_iters"] for s in stats)
    pcg = sum(s["pcg_iters"] for s in stats)
    achieved = bytes_k / (ms_k * 1e-3) / 1e9 if ms_k > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "sim steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "form": "plain FP64 GPU (explicit-velocity warm start, unbatched)",
        "newton_iters_per_step": newton / args.steps,
        "newton_iters_per_s": newton / elapsed,
        "pcg_iters_per_newton": pcg / max(newton, 1),
        "config": {"workload": f"gripper: soft ellipsoid voxelised at r={args.res} (seed {args.seed}) squeezed "
                               f"by two driven affine fingers, dt=0.005 s, {args.steps} steps",
                   "seed": args.seed, "res": args.res, "soft_vertices": G.n_soft_verts, "tets": G.n_tets,
                   "dofs": G.n_dof, "surface_triangles": G.n_tris},
        "roofline": {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "avg_launch_us": 1e3 * ms_k / max(launches, 1), "launches": launches,
                     "bytes_per_launch": bytes_k / max(launches, 1),
                     "timing_steps": args.timing_steps,
                     "share_of_step_time": ms_k * 1e-3 / t_roof},
        "autotuned": tuned,
        "phase_ms_per_step": {k: sum(s[f"ms_{k}"] for s in stats) / args.steps
                              for k in ("assemble", "pcg", "broad", "ccd", "linesearch")},
        "failed_steps": sum(1 for s in stats if s["status"] != 0),
    }
    if args.copy_probe:
        # a streaming kernel of known size (reads 256 MiB, writes 256 MiB), for scaling
        # the HBM counters of a profile
        n = 1 << 25                                  # 32 Mi doubles
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 8 * n
    if not args.no_forms:
        out["forms"] = forms(args, zema)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(sg.gripper(args.seed, r=args.res, steps=args.steps), args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
