"""Per-iterate parity at the full-size gripper (ellipsoid r = 32, seed 0: 50,664 tets,
two driven fingers): every Newton iterate of the oracle's first 8 steps (the approach
and the first contact steps, ~560 point-triangle and ~1,750 edge-edge candidates per
iterate) is fed to the library.

  * the oracle still reproduces the stored summary tests/golden/
    gripper_r32_oracle_iterates.json (energy terms to 1e-12 relative, candidate counts
    exactly), written by tests/golden/make_gripper_iterates.py from the oracle alone;
  * candidate sets bit-identical (static boxes at the iterate, r = dhat);
  * each energy term within 1e-9 relative (rounding floor as the other parity gates);
  * the total gradient norm-wise: over the soft DOFs |dg|_2 <= 1e-9 max(|g|_2, largest
    term gradient |g_k|_2) -- a converged iterate's total is a cancellation of terms
    many orders larger, so |g|_2 alone is no scale there --, over the affine DOFs the
    same plus the rounding floor of the kinematic term (below); |dg|_2 / |g|_2 and
    |g|_2 / |g_k|_2 are logged per iterate; per-term gradients on every other iterate;
  * H v within 1e-9 of |H v| on every fourth iterate (the friction term within a bound
    derived from the conditioning of its lagged weights, see fric_tol).
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


def fric_tol(R, sc, y_t):
    """Tolerance of the friction term's H v.  Its weights lambda_k = kappa |b'(d_k)| are
    taken at the lagged state, and near dhat |b'| ~ 3 (dhat - d)^2 / dhat, so a change
    delta of a lagged distance changes lambda_k by 2 delta / (dhat - d_k) relatively.
    The two sides form d_k from surface positions that differ by rounding (an affine
    body's vertex is A x0 + p), delta <= 8 eps max|x|; the tolerance is 1e-9 plus that
    bound at the nearest-to-dhat lagged pair.  When contact starts, pairs sit within
    1e-9 dhat of dhat (a few 1e-5), otherwise it is ~1e-9."""
    ids, _ = R.friction_table()
    if len(ids) == 0:
        return 1e-9
    xs = R.surface_positions(y_t)
    dhat = sc.params.dhat
    t = []
    for kind, a, b, c, d in ids:
        x12 = np.concatenate([xs[a], xs[b], xs[c], xs[d]])
        t.append(dhat - (ref.dist_pt(x12)[0] if kind == 0 else ref.dist_ee(x12)[0]))
    delta = 8.0 * np.finfo(float).eps * np.abs(xs).max()
    return 1e-9 + 2.0 * delta / max(min(t), delta)


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
    n3 = 3 * R.n_soft_verts
    # The kinematic gradient kappa_A (q - q~) of a driven body is rounding where q
    # follows its target: q and q~ (entries ~1 for A) are formed by different sums on
    # each side, each entry within 2 eps |q_i|, so the affine DOFs carry an absolute
    # floor of 4 eps kappa_A |q|_2 (kappa_A = 1e8: ~2e-7 against gradients of ~1e-5 at
    # the first iterates).  The soft DOFs keep the plain 1e-9 norm-wise gate.
    kA = max([a.kappa_A for a in sc.affines] + [0.0])

    def floor_a(y):
        return 4.0 * np.finfo(float).eps * kA * np.linalg.norm(y[n3:])
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
        dg = gg.cpu().numpy() - gr
        gn = np.linalg.norm(gr)
        gt = max(np.linalg.norm(R.ip_assemble(y, hess=False, mask=1 << k)[1]) for k in range(6))
        scale = max(gn, gt)
        rel = np.linalg.norm(dg) / gn
        rel_soft = np.linalg.norm(dg[:n3]) / scale
        worst_norm = max(worst_norm, rel_soft)
        log(f"iterate {i} (step {rc['step']}): {len(pr)} PT + {len(er)} EE candidates, "
            f"|dg|_2 / |g|_2 = {rel:.2e}, |g|_2 / largest term {gn / gt:.1e}; soft DOFs |dg|_2 / scale "
            f"{rel_soft:.2e}; affine |dg|_2 {np.linalg.norm(dg[n3:]):.2e} (floor {floor_a(y):.2e}); "
            f"barrier {tr[4]:.3e}, friction {tr[5]:.3e}")
        assert rel_soft <= 1e-9
        assert np.linalg.norm(dg[n3:]) <= 1e-9 * scale + floor_a(y)
        if i % 2 == 0:
            check_grad_terms(G, R, y, f"iterate {i}", rc["y_t"],
                             affine_floor=4.0 * np.finfo(float).eps * kA * np.abs(y[n3:]).max())
        if i % 4 == 0:
            ft = fric_tol(R, sc, rc["y_t"])
            log(f"iterate {i}: friction H v tolerance {ft:.2e}")
            check_hv(G, R, y, i, f"iterate {i}", masks=(0, 1 << 1, 1 << 4, 1 << 5), tols={1 << 5: ft})
    log(f"{len(recs)} iterates, worst norm-wise gradient error of the soft DOFs {worst_norm:.2e}")
