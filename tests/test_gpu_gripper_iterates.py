"""Per-iterate parity at the full-size gripper (ellipsoid r = 32, seed 0: 50,664 tets,
two driven fingers): every Newton iterate of the oracle's first 8 steps (the approach
and the first contact steps, ~560 point-triangle and ~1,750 edge-edge candidates per
iterate) is fed to the library.

  * the oracle still reproduces the stored summary tests/golden/
    gripper_r32_oracle_iterates.json (energy terms to 1e-12 relative, candidate counts
    exactly), written by tests/golden/make_gripper_iterates.py from the oracle alone;
  * candidate sets bit-identical (static boxes at the iterate, r = dhat);
  * each energy term within 1e-9 relative (rounding floor as the other parity gates);
  * the total gradient norm-wise, |g_gpu - g_oracle|_2 <= 1e-9 |g_oracle|_2, reported
    per iterate; per-term gradients on every other iterate;
  * H v within 1e-9 of |H v| on every fourth iterate.
"""
import json
import os

import numpy as np
import pytest

import scenegen as sg
from oracle import ref
from test_gpu_parity import check_grad_terms, check_hv, check_terms, energy_floor

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "gripper_r32_oracle_iterates.json")


def log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def zema():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_05945_amd import zema as z
    return z


@pytest.fixture(scope="module")
def iterates():
    sc = sg.gripper(0, r=32, steps=8)
    R = ref.RefScene(sc)
    R.record(True)
    R.step(8)
    return sc, R.records()


def test_gripper_iterates_follow_oracle(zema, iterates):
    sc, recs = iterates
    golden = json.load(open(GOLDEN))["iterates"]
    assert len(recs) == len(golden)
    R = ref.RefScene(sc)
    G = zema.Scene(sc)
    floor = energy_floor(sc, R)
    worst_norm = 0.0
    for i, (rc, gd) in enumerate(zip(recs, golden)):
        for S in (R, G):
            S.set_state(rc["y_t"], rc["ydot_t"], rc["kappa_lag"], rc["step"])
            S.set_kappa(rc["kappa"])
        y = rc["y_k"]
        xs = R.surface_positions(y)
        pr, er = R.candidates(xs, None)
        pg, eg = G.contact_candidates(xs, None)
        assert np.array_equal(pg.cpu().numpy(), pr) and np.array_equal(eg.cpu().numpy(), er), f"iterate {i}"
        assert (len(pr), len(er)) == (gd["n_pt"], gd["n_ee"])
        tr, gr = R.ip_assemble(y, hess=False)
        tg, gg = G.ip_assemble(y, hess=False)
        for k in range(7):
            assert tr[k] == pytest.approx(gd["terms"][k], rel=1e-12, abs=1e-300), f"oracle drift, iterate {i}"
        check_terms(tg, tr, f"iterate {i}", floor)
        rel = np.linalg.norm(gg.cpu().numpy() - gr) / np.linalg.norm(gr)
        worst_norm = max(worst_norm, rel)
        log(f"iterate {i} (step {rc['step']}): {len(pr)} PT + {len(er)} EE candidates, "
            f"|dg|_2 / |g|_2 = {rel:.2e}, barrier {tr[4]:.3e}, friction {tr[5]:.3e}")
        assert rel <= 1e-9
        if i % 2 == 0:
            check_grad_terms(G, R, y, f"iterate {i}", rc["y_t"])
        if i % 4 == 0:
            check_hv(G, R, y, i, f"iterate {i}", masks=(0, 1 << 1, 1 << 4, 1 << 5))
    log(f"{len(recs)} iterates, worst norm-wise gradient error {worst_norm:.2e}")
