"""Mixed-precision form: FP32 Hessian storage and products, FP64 everywhere else.

The energy, the gradient, the line search, the CCD bound and the convergence test
stay FP64, so they meet the FP64 gates against the oracle.  The Hessian and its
products are FP32: each 3x3 block entry carries a relative rounding of 2^-24 and a
row sums at most 27 soft neighbour blocks plus contact blocks, so H v differs from
the FP64 product by about sqrt(n_terms) * 2^-24 * |H||v| (bound n * 2^-24); the gate
is 1e-5 of max|H v| at the cube and gripper states.
Trajectories: the solution of each time step depends on the Hessian only through the
Newton path, so mixed and FP64 agree to the Newton tolerance (1e-6 h per vertex per
iteration) times the steps taken.
"""
import numpy as np
import pytest

import scenegen as sg
from gpu_helpers import scene_topology
from oracle import exact, ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def zema():
    _need_gpu()
    from paper_2311_05945_amd import zema as z
    return z


def log(*a):
    print(*a, flush=True)


def mixed(sc):
    sc.params.precision = 1
    return sc


def check_hv32(G, R, y, seed, ctx, masks):
    rng = np.random.default_rng(seed)
    worst = 0.0
    for m in masks:
        R.ip_assemble(y, mask=m)
        G.ip_assemble(y, mask=m)
        for _ in range(2):
            v = rng.normal(size=R.n_dof)
            hr = R.hessian_matvec(v)
            hg = G.hessian_matvec(v).cpu().numpy()
            scale = np.abs(hr).max()
            if scale == 0.0:
                continue
            rel = np.abs(hg - hr).max() / scale
            worst = max(worst, rel)
            assert rel <= 1e-5, f"{ctx} mask {m}: mixed H v rel err {rel:.3e}"
    return worst


def test_mixed_energy_gradient_exact_hv_fp32(zema):
    sc = mixed(sg.cube_drop())
    R = ref.RefScene(sc)
    R.record(True)
    R.step(6)
    recs = R.records()
    G = zema.Scene(sc)
    worst = 0.0
    for k, rc in enumerate(recs[::7]):
        y = rc["y_k"]
        R.set_state(rc["y_t"], rc["ydot_t"], rc["kappa_lag"], rc["step"])
        G.set_state(rc["y_t"], rc["ydot_t"], rc["kappa_lag"], rc["step"])
        R.set_kappa(rc["kappa"])
        G.set_kappa(rc["kappa"])
        tr, gr = R.ip_assemble(y, hess=False)
        tg, gg = G.ip_assemble(y, hess=False)
        assert tg[6] == pytest.approx(tr[6], rel=1e-9, abs=1e-14)
        S = np.abs(gr).max() + np.abs(R.ip_assemble(rc["y_t"], hess=False, mask=1)[1]).max()
        assert np.abs(gg.cpu().numpy() - gr).max() <= 1e-9 * S
        worst = max(worst, check_hv32(G, R, y, k, f"cube record {k}", (0, 1 << 1, 1 << 4)))
    log(f"cube mixed worst H v rel err {worst:.2e}")


def test_mixed_gripper_contact_hv(zema):
    from test_gpu_parity import gripper_contact_state
    sc = mixed(sg.gripper(0))
    R = ref.RefScene(sc)
    y, yd = gripper_contact_state(sc, R)
    R.set_state(y, yd)
    G = zema.Scene(sc)
    G.set_state(y, yd)
    worst = check_hv32(G, R, y, 3, "gripper", (0, 1 << 1, 1 << 4))
    log(f"gripper mixed worst H v rel err {worst:.2e}")


def test_mixed_trajectory_matches_fp64(zema):
    """20 cube steps in both forms: positions agree to 1e-6 m (the Newton tolerance is
    1e-6 h per iterate, h = 0.01 s here), both intersection-free, Newton counts close."""
    sc64 = sg.cube_drop()
    sc32 = mixed(sg.cube_drop())
    A = zema.Scene(sc64)
    B = zema.Scene(sc32)
    R = ref.RefScene(sc64)
    tris, edges, vb = (t.cpu().numpy() for t in A.surface_view()[:3])
    na = nb = 0
    worst = 0.0
    for k in range(4):
        sa = A.step(5)
        sb = B.step(5)
        assert all(s["status"] == 0 for s in sa + sb)
        na += sum(s["newton_iters"] for s in sa)
        nb += sum(s["newton_iters"] for s in sb)
        ya = A.get_state()[0].cpu().numpy()
        yb = B.get_state()[0].cpu().numpy()
        d = np.abs(ya - yb).max()
        worst = max(worst, d)
        xs = R.surface_positions(yb)
        assert exact.count_intersections(xs, tris, edges, vb) == 0
        log(f"steps {5 * (k + 1)}: max |y_mixed - y_fp64| {d:.3e}, newton fp64 {na} mixed {nb}")
    assert worst <= 1e-6
    assert abs(nb - na) <= 0.25 * na + 4


def test_mixed_batch_converges_intersection_free(zema):
    """An uneven batch in the mixed form (scenes running ahead of each other): every
    scene-step converges (a solve that meets non-positive curvature from FP32 rounding
    ends at its current iterate instead of failing) and stays intersection-free; the
    Newton counts stay within a few iterations of the FP64 batch."""
    seeds = (10001, 10003, 10005)
    B = zema.Scene.batch([mixed(sg.batch_scene(s)) for s in seeds])
    F = zema.Scene.batch([sg.batch_scene(s) for s in seeds])
    sb = B.step(12)
    sf = F.step(12)
    assert all(x["status"] == 0 for x in sb)
    nb = sum(x["newton_iters"] for x in sb)
    nf = sum(x["newton_iters"] for x in sf)
    y = B.get_state()[0].cpu().numpy()
    yf = F.get_state()[0].cpu().numpy()
    log(f"mixed batch: {nb} Newton iterations (FP64 {nf}), max |y - y_fp64| {np.abs(y - yf).max():.2e}")
    assert abs(nb - nf) <= 0.1 * nf + 5
    xs = B.surface_positions(y).cpu().numpy()
    for j, s in enumerate(seeds):
        xj, tris, edges, vb = scene_topology(B, j, xs)
        assert exact.count_intersections(xj, tris, edges, vb) == 0
