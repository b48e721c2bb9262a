"""Writes gripper_r32_oracle_iterates.json: per Newton iterate of the oracle's first 8
steps of the gripper workload (ellipsoid r = 32, seed 0), the step, the energy terms,
the gradient norm, the candidate counts at the iterate and the number of active pairs.

Calls only `oracle/` (and the input generator).  Run from the repository root:

    python tests/golden/make_gripper_iterates.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import scenegen as sg  # noqa: E402
from oracle import ref  # noqa: E402

STEPS = 8


def iterates(threads=0):
    """The oracle's recorded iterates of the first STEPS steps."""
    if threads:
        ref.set_threads(threads)
    R = ref.RefScene(sg.gripper(0, r=32, steps=STEPS))
    R.record(True)
    R.step(STEPS)
    return R.records()


def summary(R, rc):
    R.set_state(rc["y_t"], rc["ydot_t"], rc["kappa_lag"], rc["step"])
    R.set_kappa(rc["kappa"])
    terms, g = R.ip_assemble(rc["y_k"], hess=False)
    xs = R.surface_positions(rc["y_k"])
    pt, ee = R.candidates(xs, None)
    return {"step": int(rc["step"]), "terms": [float(t) for t in terms], "grad_norm": float(np.linalg.norm(g)),
            "n_pt": int(len(pt)), "n_ee": int(len(ee))}


def main():
    recs = iterates()
    R = ref.RefScene(sg.gripper(0, r=32, steps=STEPS))
    out = {"workload": "gripper r=32 seed 0, oracle Newton iterates of steps 0-7",
           "iterates": [summary(R, rc) for rc in recs]}
    with open(os.path.join(HERE, "gripper_r32_oracle_iterates.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"{len(recs)} iterates")


if __name__ == "__main__":
    main()
