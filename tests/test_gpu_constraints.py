"""GPU parity of the constraint energies of Sec. IV-C against the oracle.

  * springs (k |x - x_target|^2, Sec. IV-C-3) on the vertices of a free affine box
    hanging under gravity, and on soft surface vertices of the dropped cube pulled
    sideways: every step follows the oracle (same Newton counts, every DOF within
    1e-9 m), and the constraint term's energy and gradient match at the end state
    (1e-9 relative);
  * augmented Lagrangian of the kinematic energy (eq. 13) on a held box with a soft
    penalty: the same number of multiplier updates per step, multipliers within 1e-9
    relative and states within 1e-12 m of the oracle.
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def zema():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_05945_amd import zema as z
    return z


def _follow(G, R, steps, ctx, e_floor=lambda e: 0.0, g_floor=0.0):
    for k in range(steps):
        sg_ = G.step(1)[0]
        so = R.step(1)[0]
        dy = np.abs(G.get_state()[0].cpu().numpy() - R.get_state()[0]).max()
        log(f"{ctx} step {k}: newton gpu {sg_['newton_iters']} oracle {so['newton_iters']}, "
            f"al updates {sg_['al_updates']}/{so['al_updates']}, |y - y_oracle| {dy:.2e}")
        assert sg_["status"] == 0 and sg_["newton_iters"] == so["newton_iters"]
        assert sg_["al_updates"] == so["al_updates"]
        assert dy <= 1e-9
    y = R.get_state()[0]
    tr, gr = R.ip_assemble(y, hess=False, mask=1 << 3)
    tg, gg = G.ip_assemble(y, hess=False, mask=1 << 3)
    assert abs(tg[3] - tr[3]) <= 1e-9 * abs(tr[3]) + e_floor(abs(tr[3]))
    assert np.abs(gg.cpu().numpy() - gr).max() <= 1e-9 * np.abs(gr).max() + g_floor


def test_springs_on_affine_box_follow_oracle(zema):
    sc = sg.held_box(mode=sg.MODE_FREE, steps=12)
    R = ref.RefScene(sc)
    G = zema.Scene(sc)
    xs0 = R.surface_positions(R.get_state()[0])
    n = len(xs0)
    rng = np.random.default_rng(0)
    k = rng.uniform(100.0, 300.0, n)
    R.set_springs(np.arange(n), k, xs0)
    G.set_springs(np.arange(n), k, xs0)
    _follow(G, R, 12, "box")


def test_springs_on_soft_vertices_follow_oracle(zema):
    sc = sg.cube_drop()
    R = ref.RefScene(sc)
    G = zema.Scene(sc)
    tris, edges, vb = R.surface()
    xs0 = R.surface_positions(R.get_state()[0])
    soft = np.nonzero(vb == 0)[0][::7]
    tgt = xs0[soft] + np.array([0.004, 0.0, -0.002])
    k = np.full(len(soft), 50.0)
    R.set_springs(soft, k, tgt)
    G.set_springs(soft, k, tgt)
    _follow(G, R, 8, "cube")


def test_kinematic_multiplier_follows_oracle(zema):
    sc = sg.held_box(kappa_A=1e3, steps=6)
    R = ref.RefScene(sc)
    G = zema.Scene(sc)
    tol = 5e-11
    R.kinematic_al(tol, 12)
    G.kinematic_al(tol, 12)
    _follow(G, R, 6, "held box")
    lr = R.kinematic_al(tol, 12)
    lg = G.kinematic_al(tol, 12)
    log(f"multiplier gpu {lg[0][:3]} oracle {lr[0][:3]}")
    assert np.abs(lg - lr).max() <= 1e-9 * np.abs(lr).max() and np.abs(lr).max() > 0


@pytest.mark.parametrize("rail", ["fixed", "free"])
def test_prismatic_joint_follows_oracle(zema, rail):
    """A box sliding along a rail (Sec. IV-C-2 joint, axis x): with a fixed rail the
    joint acts on the box alone; with a free rail its 24x24 Gauss-Newton Hessian couples
    the two bodies' DOFs (blocks between them in the contact CSR)."""
    sc = sg.slider_scene(steps=10)
    if rail == "free":
        sc.affines[0].mode = sg.MODE_FREE
    R = ref.RefScene(sc)
    G = zema.Scene(sc)
    kappa, L, eps = 10.0, 0.1, np.finfo(float).eps
    for S in (R, G):
        S.set_prismatic_joints([[1, 0]], [[1.0, 0.0, 0.0]], [kappa])
    # a joint that holds leaves residuals R near the rounding of positions of size L:
    # |dR| <~ 16 eps L, so |dE| <= 2 sqrt(kappa E) 16 eps L and |dg| <~ 2 kappa 16 eps L
    _follow(G, R, 10, f"slider ({rail} rail)", e_floor=lambda e: 2 * np.sqrt(kappa * e) * 16 * eps * L,
            g_floor=2 * kappa * 16 * eps * L)
    y = R.get_state()[0]
    rng = np.random.default_rng(1)
    R.ip_assemble(y, mask=1 << 3)
    G.ip_assemble(y, mask=1 << 3)
    for _ in range(3):
        v = rng.normal(size=len(y))
        hr = R.hessian_matvec(v)
        hg = G.hessian_matvec(v).cpu().numpy()
        assert np.abs(hg - hr).max() <= 1e-9 * np.abs(hr).max()
