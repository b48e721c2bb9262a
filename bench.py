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


def cpu_baseline(scene, seconds, gpu_stats, max_steps=20):
    """The oracle as it stands, timed on the host cores on the same steps as the GPU:
    the first steps of the same trajectory until `seconds` of CPU time have been spent
    (at least one step), with every core, then the first step on one thread.  The GPU
    figure for the same steps comes from the timed run's per-step wall times."""
    from oracle import ref
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    used = ref.set_threads(threads)
    R = ref.RefScene(scene)
    t = 0.0
    n = 0
    newton = 0
    while n < min(max_steps, len(gpu_stats)) and (n == 0 or t < seconds):
        t0 = time.perf_counter()
        st = R.step(1)[0]
        t += time.perf_counter() - t0
        n += 1
        newton += st["newton_iters"]
        log(f"cpu oracle step {n}: {t:.1f} s total, newton {st['newton_iters']}, pcg {st['pcg_iters']}")
    gpu_t = sum(x["ms_total"] for x in gpu_stats[:n]) * 1e-3
    gpu_newton = sum(x["newton_iters"] for x in gpu_stats[:n])
    ref.set_threads(1)
    R1 = ref.RefScene(scene)
    t1 = time.perf_counter()
    st1 = R1.step(1)[0]
    t1 = time.perf_counter() - t1
    ref.set_threads(threads)
    log(f"cpu oracle, one thread: step 1 in {t1:.2f} s")
    return {"value": n / t, "unit": "sim steps/s", "cores": used, "kind": "oracle",
            "sample": f"steps 0-{n - 1} of the timed trajectory ({newton} Newton iterations, {t:.1f} s on {used} "
                      f"threads; these early steps include the contact-free approach of the fingers)",
            "newton_iters_per_s": newton / t,
            "gpu_same_steps": {"steps_per_s": n / gpu_t if gpu_t > 0 else None,
                               "newton_iters_per_s": gpu_newton / gpu_t if gpu_t > 0 else None,
                               "newton_iters": gpu_newton},
            "one_thread": {"steps_per_s": 1.0 / t1, "newton_iters_per_s": st1["newton_iters"] / t1,
                           "sample": "step 0 of the same trajectory"}}


def cube_drop_leg(zema):
    """The soft-cube drop (384 tets on a fixed slab, 20 steps of 0.01 s): the GPU plain
    form against the oracle on every core, same steps, same tolerance."""
    import torch

    import scenegen as sg
    from oracle import ref
    sc = sg.cube_drop()
    G = zema.Scene(sc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sg_ = G.step(sc.n_steps)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    used = ref.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    R = ref.RefScene(sc)
    t0 = time.perf_counter()
    so = R.step(sc.n_steps)
    tr = time.perf_counter() - t0
    ng = sum(x["newton_iters"] for x in sg_)
    nr = sum(x["newton_iters"] for x in so)
    dy = float(abs(G.get_state()[0].cpu().numpy() - R.get_state()[0]).max())
    log(f"cube drop: gpu {sc.n_steps / tg:.1f} steps/s ({ng} Newton), oracle {sc.n_steps / tr:.1f} steps/s ({nr} Newton)")
    return {"workload": "soft cube 0.1 m (384 tets) dropped from 5 mm onto a fixed slab, dt=0.01 s, 20 steps",
            "gpu": {"steps_per_s": sc.n_steps / tg, "newton_iters_per_step": ng / sc.n_steps,
                    "newton_iters_per_s": ng / tg},
            "oracle": {"steps_per_s": sc.n_steps / tr, "newton_iters_per_step": nr / sc.n_steps,
                       "newton_iters_per_s": nr / tr, "cores": used},
            "max_position_diff_m": dy, "failed_steps": sum(1 for x in sg_ if x["status"] != 0)}


def garment_leg(zema):
    """The garment dropped onto a fixed cone (Baraff-Witkin membrane, 121 vertices, 200
    triangles, dt = 0.005 s, 20 steps): the GPU plain form against the oracle on every
    core, same steps, same tolerance."""
    import torch

    import scenegen as sg
    from oracle import ref
    sc = sg.garment_on_cone(gap=2e-3, steps=20)
    sc.params.dt = 0.005
    G = zema.Scene(sc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sg_ = G.step(sc.n_steps)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    used = ref.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    R = ref.RefScene(sc)
    t0 = time.perf_counter()
    so = R.step(sc.n_steps)
    tr = time.perf_counter() - t0
    ng = sum(x["newton_iters"] for x in sg_)
    nr = sum(x["newton_iters"] for x in so)
    dy = float(abs(G.get_state()[0].cpu().numpy() - R.get_state()[0]).max())
    log(f"garment: gpu {sc.n_steps / tg:.1f} steps/s ({ng} Newton), oracle {sc.n_steps / tr:.1f} steps/s ({nr} Newton)")
    return {"workload": "Baraff-Witkin garment 0.3 m (10x10 quads, 200 triangles) dropped 2 mm onto a fixed cone, "
                        "dt=0.005 s, 20 steps",
            "gpu": {"steps_per_s": sc.n_steps / tg, "newton_iters_per_step": ng / sc.n_steps,
                    "newton_iters_per_s": ng / tg},
            "oracle": {"steps_per_s": sc.n_steps / tr, "newton_iters_per_step": nr / sc.n_steps,
                       "newton_iters_per_s": nr / tr, "cores": used},
            "max_position_diff_m": dy, "failed_steps": sum(1 for x in sg_ if x["status"] != 0)}


def precision_leg(zema, res, steps, seed):
    """The gripper at a finer grid (r = 64 by default): the mixed form (FP32 elastic
    Hessian and products) and the FP64 form on the GPU and the oracle, the first `steps`
    steps; per step the energy at each path's own end state, the norm of the gradient
    left at that state (the converged step's residual force) relative to the gradient
    norm at the step's start, and the largest position difference."""
    import numpy as np
    import torch

    import scenegen as sg
    from oracle import ref
    out = {"workload": f"gripper, ellipsoid voxelised at r={res} (seed {seed}), first {steps} steps", "steps": []}
    paths = {}
    for name, prec in (("fp64", 0), ("mixed", 1)):
        sc = sg.gripper(seed, r=res, steps=steps)
        sc.params.precision = prec
        G = zema.Scene(sc)
        if name == "fp64":
            out.update(tets=G.n_tets, soft_vertices=G.n_soft_verts, dofs=G.n_dof)
        rec = []
        torch.cuda.synchronize()
        t = 0.0
        for k in range(steps):
            g0 = float(torch.linalg.norm(G.ip_assemble(G.get_state()[0], hess=False)[1]))
            t0 = time.perf_counter()
            st = G.step(1)[0]
            torch.cuda.synchronize()
            t += time.perf_counter() - t0
            y = G.get_state()[0]
            terms, g = G.ip_assemble(y, hess=False)
            rec.append((y.cpu().numpy(), float(terms[6]), float(torch.linalg.norm(g)) / g0, st["newton_iters"]))
        paths[name] = (rec, t)
        log(f"precision leg {name}: {steps} steps in {t:.2f} s")
    used = ref.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    R = ref.RefScene(sg.gripper(seed, r=res, steps=steps))
    rec = []
    t = 0.0
    for k in range(steps):
        g0 = float(np.linalg.norm(R.ip_assemble(R.get_state()[0], hess=False)[1]))
        t0 = time.perf_counter()
        st = R.step(1)[0]
        t += time.perf_counter() - t0
        y = R.get_state()[0]
        terms, g = R.ip_assemble(y, hess=False)
        rec.append((y, float(terms[6]), float(np.linalg.norm(g)) / g0, st["newton_iters"]))
        log(f"precision leg oracle step {k}: {t:.1f} s")
    paths["oracle"] = (rec, t)
    for k in range(steps):
        (yf, ef, gf, nf), (ym, em, gm, nm), (yo, eo, go, no) = (paths[n][0][k] for n in ("fp64", "mixed", "oracle"))
        out["steps"].append({
            "step": k, "newton": {"fp64": nf, "mixed": nm, "oracle": no},
            "residual_grad_norm_rel_to_step_start": {"fp64": gf, "mixed": gm, "oracle": go},
            "mixed_vs_fp64": {"energy_rel": abs(em - ef) / abs(ef), "max_position_m": float(np.abs(ym - yf).max())},
            "mixed_vs_oracle": {"energy_rel": abs(em - eo) / abs(eo), "max_position_m": float(np.abs(ym - yo).max())},
            "fp64_vs_oracle": {"energy_rel": abs(ef - eo) / abs(eo), "max_position_m": float(np.abs(yf - yo).max())}})
    out["seconds"] = {n: paths[n][1] for n in paths}
    out["oracle_cores"] = used
    return out


def hbm_traffic(kernel, source_files):
    """HBM bytes per launch of `kernel` from the committed counter profile, or None when
    the profile is missing or a source of the kernel changed since it was taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "hbm_counters_gripper.md")
    if not os.path.exists(prof):
        return None
    h = hashlib.sha256()
    for f in source_files:
        h.update(open(os.path.join(ROOT, "paper_2311_05945_amd", "csrc", f), "rb").read())
    sha = h.hexdigest()
    for line in open(prof):
        f = line.split()
        if len(f) == 6 and f[0] == "traffic" and f[1] == kernel and f[5] == sha:
            return float(f[3])
    return None


def run_form(zema, scenes, steps, batched, learned=None, mixed=False, chunk=5, group_chunk=10, tag="",
             groups=GROUPS, newton_max=0, warm_fit=-1):
    """Steps every scene `steps` times; returns (wall seconds, stats list, [intersecting
    edge-triangle pairs, inverted tets, uncertain pairs] at the end: the last are pairs
    the filtered predicates could not decide, touching or coplanar to rounding, which
    only an exact check resolves)."""
    import copy

    import torch
    scenes = [copy.deepcopy(sc) for sc in scenes]
    for sc in scenes:
        sc.params.precision = 1 if mixed else 0
        sc.params.warm_start = 1 if learned is not None else 0
        if newton_max:
            sc.params.newton_max = newton_max
    # batched: the scenes in GROUPS batch objects on as many streams, stepped together
    # (zema_step_group); within a call every scene starts its next step as soon as it
    # has converged
    if batched:  # as zema.batch_group: similar sizes (largest first, dealt round-robin), one stream each
        import torch as _t
        order = sorted(range(len(scenes)), key=lambda i: -sum(len(b.rest_pos) for b in scenes[i].softs))
        objs = []
        for g in range(groups):
            part = [scenes[i] for i in order[g::groups]]
            if part:
                objs.append(zema.Scene.batch(part, stream=_t.cuda.Stream()))
                log(f"form {tag}: batch object {len(objs)} of {len(part)} scenes created")
    else:
        objs = [zema.Scene(sc) for sc in scenes]
    for o in objs:
        if learned is not None:
            o.set_mlp(learned)
            if warm_fit >= 0:
                o.tune(zema.TUNE_WARM_FIT, warm_fit)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    if batched:
        done = 0
        while done < steps:
            n = min(group_chunk, steps - done)
            for st in zema.step_group(objs, n):
                stats += st
            done += n
            log(f"form {tag}: {done}/{steps} steps of {len(scenes)} scenes, {time.perf_counter() - t0:.1f} s")
    for i, o in enumerate(objs if not batched else []):
        done = 0
        while done < steps:
            n = min(chunk, steps - done)
            stats += o.step(n)
            done += n
        if (i + 1) % 8 == 0:
            log(f"form {tag}: {i + 1}/{len(objs)} scenes, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    inter = [0, 0, 0]  # intersecting (edge, triangle) pairs, inverted tets, pairs the filter left uncertain
    for o in objs:
        ni, nv, nu, _ = o.intersection_count(o.get_state()[0], cap=0)
        inter[0] += ni
        inter[1] += nv
        inter[2] += nu
    return t, stats, inter


def forms(args, zema):
    """The batched, learned and mixed-precision forms against the plain form, on uneven
    grasp scenes at the same Newton tolerance.  The unbatched forms (plain, learned) run
    one scene after the other, on the first `form_plain_scenes` scenes when that is set
    (their rate per scene-step does not depend on how many scenes run)."""
    import numpy as np

    import scenegen as sg
    seeds = list(range(args.form_seed, args.form_seed + args.form_scenes))
    t0 = time.perf_counter()
    scenes = [sg.batch_scene(s, steps=args.form_steps) for s in seeds]
    log(f"forms: {len(scenes)} scenes generated in {time.perf_counter() - t0:.1f} s, "
        f"{sum(sum(len(b.tets) for b in sc.softs) for sc in scenes)} tets")
    n_plain = args.form_plain_scenes if args.form_plain_scenes > 0 else len(scenes)
    mlp = None
    if os.path.exists(args.mlp):
        mlp = zema.Mlp(np.load(args.mlp))
    out = {"sample": f"{len(seeds)} uneven grasp scenes (seeds {seeds[0]}-{seeds[-1]}), {args.form_steps} steps "
                     f"each from rest, dt=0.005 s, Newton tol 1e-6 dt",
           "unbatched_sample": f"first {n_plain} scenes",
           "newton_max": args.form_newton_max,
           "network": os.path.basename(args.mlp) if mlp is not None else None,
           "warm_fit": args.warm_fit if args.warm_fit >= 0 else "library default (2: per-body mean)",
           "batched_steps_per_call": args.form_group_chunk,
           "batched_as": f"{args.form_groups} batch objects of similar size on as many HIP streams, stepped together "
                         f"(zema_step_group); plain: one scene object after the other"}
    cases = [("plain", False, None, False), ("batched", True, None, False)]
    if mlp is not None:
        cases += [("learned", False, mlp, False), ("batched_learned", True, mlp, False),
                  ("batched_learned_mixed", True, mlp, True)]
    if args.form_cases:
        keep = args.form_cases.split(",")
        cases = [c for c in cases if c[0] in keep]
    # untimed warm-up of the grouped batch path (streams, host threads, first launches)
    run_form(zema, scenes[:min(8, len(scenes))], 2, True, tag="warm-up")
    for name, batched, learned, mixed in cases:
        sub = scenes if batched else scenes[:n_plain]
        t, st, inter = run_form(zema, sub, args.form_steps, batched, learned, mixed, tag=name, warm_fit=args.warm_fit,
                                groups=args.form_groups, newton_max=args.form_newton_max,
                                group_chunk=args.form_group_chunk)
        total = len(sub) * args.form_steps
        newton = sum(x["newton_iters"] for x in st)
        out[name] = {"scenes": len(sub), "steps_per_s": total / t, "newton_iters_per_step": newton / total,
                     "wall_s": t, "intersections": inter[0] + inter[1], "uncertain_pairs": inter[2],
                     "failed_steps": sum(1 for x in st if x["status"] != 0),
                     "learned_start_kept": (sum(x["warm_learned"] for x in st) / total) if learned else None}
        log(f"form {name}: {total / t:.2f} scene-steps/s, newton/step {newton / total:.2f}, "
            f"intersections {inter[0] + inter[1]}, uncertain {inter[2]}")
    if "plain" in out:
        base = out["plain"]["steps_per_s"]
        for name, *_ in cases:
            if name != "plain":
                out[name]["speedup_vs_plain"] = out[name]["steps_per_s"] / base
    return out


def warm_analysis(zema, seed0, n_scenes, steps, mlp_path, fits=(0, 1, 2)):
    """The learned initial guess against the explicit one on held-out uneven scenes:
    from the same state, per step, the distance of each proposal (soft vertices; the
    explicit x + h v, the network's x + h v + s out) to the converged state, the Newton
    iterations of a step started from each (the library's filtered start, the learned
    one kept when its energy is not higher) and whether the learned start was kept.
    The learned start runs once per setting of the per-body fit of the network's
    correction (0 as is, 1 affine fit, 2 mean)."""
    import numpy as np
    import torch

    import scenegen as sg
    mlp = zema.Mlp(np.load(mlp_path))
    rows = []
    for s in range(seed0, seed0 + n_scenes):
        sc = sg.batch_scene(s, steps=steps)
        sc.params.newton_max = 2000
        A = zema.Scene(sc)
        Ls = []
        for f in fits:
            scl = sg.batch_scene(s, steps=steps)
            scl.params.newton_max = 2000
            scl.params.warm_start = 1
            L = zema.Scene(scl)
            L.set_mlp(mlp)
            L.tune(zema.TUNE_WARM_FIT, f)
            Ls.append(L)
        h = sc.params.dt
        n = A.n_soft_verts
        for k in range(steps):
            y, yd, kappa, step = A.get_state()
            out = mlp.forward(A.features())
            ye = (y[:3 * n] + h * yd[:3 * n]).reshape(-1, 3)
            yl = ye + h * 0.05 * out.double()
            sl = []
            for L in Ls:
                L.set_state(y, yd, kappa, step)
                sl.append(L.step(1)[0])
            se = A.step(1)[0]
            ys = A.get_state()[0][:3 * n].reshape(-1, 3)
            de = float(torch.linalg.norm(ye - ys, dim=1).pow(2).mean().sqrt())
            dl = float(torch.linalg.norm(yl - ys, dim=1).pow(2).mean().sqrt())
            rows.append([se["newton_iters"], de, dl, se["n_pt_active"] > 0,
                         se["status"] == 0 and all(x["status"] == 0 for x in sl)]
                        + [x["newton_iters"] for x in sl] + [x["warm_learned"] for x in sl])
        log(f"warm analysis: scene {s} done")
    a = np.array(rows, dtype=float)
    ne, de, dl, contact, ok = a[:, :5].T
    nf = len(fits)
    nl, kept = a[:, 5:5 + nf].T, a[:, 5 + nf:].T

    def part(m, j):
        return {"steps": int(m.sum()), "newton_explicit": float(ne[m].mean()), "newton_learned": float(nl[j][m].mean()),
                "rms_dist_explicit_m": float(de[m].mean()), "rms_dist_learned_m": float(dl[m].mean()),
                "learned_closer": float((dl[m] < de[m]).mean())} if m.any() else None
    names = {0: "as_is", 1: "affine_fit", 2: "mean"}
    res = {"sample": f"{n_scenes} held-out uneven scenes (seeds {seed0}-{seed0 + n_scenes - 1}), {steps} steps",
           "all_converged": bool(ok.all()),
           "note": "rms distances are of the network's own proposal (as is)"}
    for j, f in enumerate(fits):
        res[names[f]] = {"all": part(np.ones(len(a), bool), j), "contact": part(contact == 1, j),
                         "free": part(contact == 0, j), "learned_kept": part(kept[j] == 1, j),
                         "learned_rejected": part(kept[j] == 0, j), "kept_fraction": float(kept[j].mean())}
    return res


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
    ap.add_argument("--lanes", type=int, default=0, help="lanes per soft row of the PCG iteration (0: library default)")
    ap.add_argument("--no-graph", action="store_true", help="launch PCG kernels individually")
    ap.add_argument("--copy-probe", action="store_true", help="run a 256 MiB device copy (counter scaling)")
    ap.add_argument("--form-scenes", type=int, default=32)
    ap.add_argument("--form-steps", type=int, default=16)
    ap.add_argument("--form-seed", type=int, default=10000)
    ap.add_argument("--form-cases", default="", help="comma-separated subset of the forms (default: all)")
    ap.add_argument("--form-groups", type=int, default=GROUPS, help="batch objects of the batched forms")
    ap.add_argument("--form-group-chunk", type=int, default=10,
                    help="steps per call of the batched forms (scenes run ahead of each other within a call)")
    ap.add_argument("--form-newton-max", type=int, default=1000,
                    help="Newton iteration cap of the uneven scenes (contact onset can need several hundred)")
    ap.add_argument("--form-plain-scenes", type=int, default=0,
                    help="run the unbatched forms on the first K scenes only (0: all)")
    ap.add_argument("--mlp", default=os.path.join(ROOT, "paper_2311_05945_amd", "warm_mlp.npy"))
    ap.add_argument("--warm-fit", type=int, default=-1, choices=(-1, 0, 1, 2),
                    help="per-body fit of the network's correction in the learned forms (-1: library default)")
    ap.add_argument("--no-legs", action="store_true", help="skip the cube-drop and precision legs")
    ap.add_argument("--warm-analysis", type=int, default=0, metavar="N",
                    help="only run the learned-start analysis on N held-out scenes (--form-steps steps each)")
    ap.add_argument("--precision-res", type=int, default=64)
    ap.add_argument("--precision-steps", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import scenegen as sg
    from paper_2311_05945_amd import zema

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.warm_analysis:
        print(json.dumps({"warm_analysis": warm_analysis(zema, args.form_seed, args.warm_analysis, args.form_steps,
                                                         args.mlp)}))
        return
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
    if args.lanes:
        G.tune(zema.TUNE_SPMV_LANES, args.lanes)
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
    # timed kernels (PCG: every replayed chunk of 16 iterations; timed solves check
    # convergence after every chunk, so this pass is not part of the throughput figure;
    # elastic assembly: the per-tet kernel and its two gathers)
    G.kernel_timer(group, True)
    G.kernel_timer(GROUPS_T["tet"], True)
    torch.cuda.synchronize()
    tr0 = time.perf_counter()
    rstats = G.step(args.timing_steps)
    torch.cuda.synchronize()
    t_roof = time.perf_counter() - tr0
    ms_k, launches, bytes_k = G.kernel_time(group)
    ms_a, launches_a, bytes_a = G.kernel_time(GROUPS_T["tet"])
    log(f"roofline pass: {args.timing_steps} steps, {launches} launches of {args.timer}, {ms_k:.1f} ms; "
        f"{launches_a} elastic assemblies, {ms_a:.2f} ms")
    traffic = None
    kname = {"spmv": f"pcg_cg_kernel<double,{G.spmv_lanes()},false>"}.get(args.timer, args.timer)
    if args.timer == "spmv" and not G.params.precision:
        traffic = hbm_traffic(kname, ["k_sparse.hip", "common.hpp"])
    traffic_a = None if G.params.precision else hbm_traffic("elastic_assembly<double>",
                                                            ["k_elastic.hip", "material.hpp", "common.hpp"])
    newton = sum(s["newton_iters"] for s in stats)
    pcg = sum(s["pcg_iters"] for s in stats)
    achieved = bytes_k / (ms_k * 1e-3) / 1e9 if ms_k > 0 else 0.0
    achieved_a = bytes_a / (ms_a * 1e-3) / 1e9 if ms_a > 0 else 0.0
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
                     "share_of_step_time": ms_k * 1e-3 / t_roof,
                     "note": "one PCG iteration per launch; at this system size the launch is limited by "
                             "its dependent gathers and dispatch latency, not by HBM bandwidth"},
        "assembly_roofline": {"kernel": "elastic assembly (tet_assemble_kernel + gather_grad_soft_kernel + "
                                        "gather_hess_kernel)",
                              "bound": "hbm", "achieved": achieved_a, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": achieved_a / HBM_PEAK_GBS, "traffic": traffic_a,
                              "avg_launch_us": 1e3 * ms_a / max(launches_a, 1), "launches": launches_a,
                              "bytes_per_launch": bytes_a / max(launches_a, 1),
                              "algorithmic_bytes": "320 B per tet (ids, Dm^-1, volume, BSR share, positions, "
                                                   "gradient)"},
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
    if not args.no_legs:
        out["cube_drop"] = cube_drop_leg(zema)
        try:
            out["garment_drop"] = garment_leg(zema)
        except zema.ZemaError as e:  # reported, not fatal to the bench line
            out["garment_drop"] = {"error": str(e)}
        if args.precision_steps > 0:
            out["precision"] = precision_leg(zema, args.precision_res, args.precision_steps, args.seed)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(sg.gripper(args.seed, r=args.res, steps=args.steps), args.cpu_seconds,
                                           stats)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
