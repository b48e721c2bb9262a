"""Step-by-step comparison of the HIP library and the oracle on the gripper workload.

Usage (GPU required): python tests/trajectory_compare.py [steps] [seed] [res]
Both sides start from the same initial state and take one time step at a time; the
line per step gives Newton / PCG iterations, line-search backtracks, CCD bound,
barrier stiffness, minimum distance, active pairs, wall time and max |y_gpu - y_oracle|.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import scenegen as sg  # noqa: E402
from oracle import ref  # noqa: E402
from paper_2311_05945_amd import zema  # noqa: E402


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 16
    seed = int(sys.argv[2]) if len(sys.argv) > 2 else 0
    res = int(sys.argv[3]) if len(sys.argv) > 3 else 32
    sc = sg.gripper(seed, r=res)
    G = zema.Scene(sc)
    ref.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    R = ref.RefScene(sc)
    for k in range(n):
        t0 = time.time(); a = G.step(1)[0]; tg = time.time() - t0
        t0 = time.time(); b = R.step(1)[0]; tr = time.time() - t0
        dy = np.abs(G.get_state()[0].cpu().numpy() - R.get_state()[0]).max()
        print(f"step {k:3d} gpu: nw {a['newton_iters']:3d} pcg {a['pcg_iters']:5d} ls {a['ls_backtracks']:3d} "
              f"a {a['alpha_ccd_min']:.3f} k {a['kappa']:.3e} dmin {a['d_min']:.3e} act {a['n_pt_active']} "
              f"fr {a['n_ee_active']} {tg * 1e3:.0f}ms | ora: nw {b['newton_iters']:3d} pcg {b['pcg_iters']:5d} "
              f"ls {b['ls_backtracks']:3d} a {b['alpha_ccd_min']:.3f} k {b['kappa']:.3e} dmin {b['d_min']:.3e} "
              f"act {b['n_pt_active']}+{b['n_ee_active']} {tr:.1f}s | |dy| {dy:.2e}", flush=True)


if __name__ == "__main__":
    main()
