"""GPU checks of the C-ABI's topology, Hessian export and candidate-set modes.

* zema_surface_view: the triangles, edges and surface-vertex bodies that the pair
  lists index equal the oracle's topology (the primitives of the contact set C of
  Sec. III eq. 4); each vertex's source maps to its DOFs.
* zema_hessian_bsr: the exported block rows reproduce zema_hessian_matvec and the
  oracle's H v (eqs. 6-8), symmetric, on cube iterates, the full-size gripper state
  and a free affine body in contact; the mixed form exports its FP32 blocks.
* zema_ip_assemble without ZEMA_REBUILD evaluates the stored candidate set: a swept
  set of [y, y + p] gives the oracle's energies at y + a p, an empty stored set gives
  no barrier energy.
* Mixed-form PCG: the reported residual is the true FP64 residual of the exported
  FP32 operator and meets the tolerance.
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


def bsr_matvec(rp, col, val, v):
    """y = H v from exported block rows, in FP64 numpy."""
    rp = rp.cpu().numpy(); col = col.cpu().numpy(); val = val.cpu().numpy()
    n = len(rp) - 1
    V = v.reshape(-1, 3)
    rows = np.repeat(np.arange(n), np.diff(rp))
    prod = np.einsum("kij,kj->ki", val, V[col])
    out = np.zeros((n, 3))
    np.add.at(out, rows, prod)
    return out.ravel()


def check_bsr(G, hv, n_dof, rng, ctx):
    rp, col, val = G.hessian_bsr()
    n = n_dof // 3
    assert rp.shape[0] == n + 1 and rp[0].item() == 0 and rp[-1].item() == col.shape[0]
    rpn, cn = rp.cpu().numpy(), col.cpu().numpy()
    for r in range(n):                                  # ascending columns within each row
        assert np.all(np.diff(cn[rpn[r]:rpn[r + 1]]) > 0)
    # symmetric: block (r, c) is the transpose of block (c, r), up to the rounding of
    # entries (i, j) and (j, i) of a local block formed in different orders
    keys = {(r, c): k for r in range(n) for k, c in zip(range(rpn[r], rpn[r + 1]), cn[rpn[r]:rpn[r + 1]])}
    vn = val.cpu().numpy().astype(np.float64)
    big = np.abs(vn).max()
    eps = np.finfo(val.cpu().numpy().dtype).eps
    for (r, c), k in list(keys.items())[::7]:
        assert (c, r) in keys
        assert np.abs(vn[k] - vn[keys[(c, r)]].T).max() <= 64 * eps * big, (r, c)
    worst = 0.0
    for _ in range(3):
        v = rng.normal(size=n_dof)
        a = bsr_matvec(rp, col, val, v)
        b = G.hessian_matvec(v).cpu().numpy()
        c = hv(v)
        scale = np.abs(c).max()
        worst = max(worst, np.abs(a - c).max() / scale)
        assert np.abs(a - b).max() <= 1e-12 * scale, ctx
        assert np.abs(a - c).max() <= 1e-9 * scale, ctx
    log(f"{ctx}: {col.shape[0]} blocks, BSR product vs oracle {worst:.2e}")


def test_surface_view_matches_oracle(zema):
    for sc in (sg.cube_drop(), sg.box_on_cube(), sg.gripper(0, r=16)):
        R = ref.RefScene(sc)
        G = zema.Scene(sc)
        tris, edges, vb, vs = (t.cpu().numpy() for t in G.surface_view())
        tr, er, vr = R.surface()
        assert np.array_equal(tris, tr) and np.array_equal(edges, er) and np.array_equal(vb, vr)
        y = R.get_state()[0]
        xs = R.surface_positions(y)
        soft = vs >= 0
        assert np.array_equal(xs[soft], y[:3 * R.n_soft_verts].reshape(-1, 3)[vs[soft]])
        n_soft_bodies = len(sc.softs)
        assert np.array_equal(vb[~soft], n_soft_bodies - 1 - vs[~soft])   # -(1 + affine body)
        log(f"{sc.name}: {len(tris)} tris, {len(edges)} edges, {soft.sum()} soft surface vertices")


@pytest.fixture(scope="module")
def cube_iterates():
    sc = sg.cube_drop()
    R = ref.RefScene(sc)
    R.record(True)
    R.step(6)
    return sc, R.records()


def test_hessian_bsr_cube_and_gripper(zema, cube_iterates):
    sc, recs = cube_iterates
    R = ref.RefScene(sc)
    G = zema.Scene(sc)
    rng = np.random.default_rng(1)
    for i, rc in enumerate(recs[::4]):
        for S in (R, G):
            S.set_state(rc["y_t"], rc["ydot_t"], rc["kappa_lag"], rc["step"])
            S.set_kappa(rc["kappa"])
            S.ip_assemble(rc["y_k"])
        check_bsr(G, R.hessian_matvec, R.n_dof, rng, f"cube iterate {i}")
    gs = sg.gripper(0, r=16)
    R = ref.RefScene(gs)
    G = zema.Scene(gs)
    y, yd, _, _ = R.get_state()
    n3 = 3 * R.n_soft_verts
    y = y.copy()
    for k, f in enumerate(gs.affines):      # fingers half a d-hat from the object
        side = -1.0 if f.rest_pos[:, 0].mean() < 0 else 1.0
        y[n3 + 12 * k] -= side * 1.5 * gs.params.dhat
    R.set_state(y, yd); G.set_state(y, yd)
    assert R.ip_assemble(y)[0][4] > 0
    G.ip_assemble(y)
    check_bsr(G, R.hessian_matvec, R.n_dof, rng, "gripper r=16")


def test_hessian_bsr_free_body_and_capacity(zema):
    sc = sg.box_on_cube()
    R = ref.RefScene(sc)
    R.record(True)
    R.step(5)
    rc = R.records()[-1]
    G = zema.Scene(sc)
    for S in (R, G):
        S.set_state(rc["y_t"], rc["ydot_t"], rc["kappa_lag"], rc["step"])
        S.set_kappa(rc["kappa"])
        S.ip_assemble(rc["y_k"])
    check_bsr(G, R.hessian_matvec, R.n_dof, np.random.default_rng(2), "box on cube")
    from paper_2311_05945_amd.zema import lib, I64, E_CAPACITY
    import ctypes as C
    n = I64()
    assert lib().zema_hessian_bsr(G.h, None, None, None, 0, C.byref(n)) == E_CAPACITY and n.value > 0


def test_stored_candidate_mode(zema, cube_iterates):
    sc, recs = cube_iterates
    rc = recs[-1]
    R = ref.RefScene(sc)
    G = zema.Scene(sc)
    for S in (R, G):
        S.set_state(rc["y_t"], rc["ydot_t"], rc["kappa_lag"], rc["step"])
        S.set_kappa(rc["kappa"])
    y = rc["y_k"]
    p = np.zeros_like(y)
    p[1::3] = -2e-4
    p += np.random.default_rng(3).normal(scale=2e-5, size=p.shape)
    a = G.ccd_max_step(y, p)            # stores the swept candidate set of [y, y + p]
    ya = y + 0.5 * a * p
    t_stored, g_stored = G.ip_assemble(ya, rebuild=False)
    t_rebuilt, g_rebuilt = G.ip_assemble(ya, rebuild=True)
    t_ref, g_ref = R.ip_assemble(ya)
    log(f"stored swept set: barrier {t_stored[4]:.6e}, rebuilt {t_rebuilt[4]:.6e}, oracle {t_ref[4]:.6e}")
    assert t_ref[4] > 0
    for k in range(6):
        assert abs(t_stored[k] - t_ref[k]) <= 1e-9 * abs(t_ref[k]) + 1e-12 * abs(t_ref[6])
    scale = np.abs(g_ref).max()
    assert np.abs(g_stored.cpu().numpy() - g_ref).max() <= 1e-9 * scale
    # an empty stored set: no pair is active, so no barrier energy
    xs = G.surface_positions(ya)
    vb = G.surface_view()[2]
    far = xs.clone()
    far[vb == 0, 1] += 10.0                   # the soft body 10 m above the slab
    pt, ee = G.contact_candidates(far, None, 0.0)
    assert pt.shape[0] == 0 and ee.shape[0] == 0
    t_empty, _ = G.ip_assemble(ya, grad=False, hess=False, rebuild=False)
    assert t_empty[4] == 0.0 and t_empty[7] == float("inf")
    t_again, _ = G.ip_assemble(ya, grad=False, hess=False, rebuild=True)
    assert t_again[4] == t_rebuilt[4]


def test_mixed_pcg_reports_true_residual(zema):
    sc = sg.gripper(0, r=16, precision=sg.PREC_MIXED)
    G = zema.Scene(sc)
    G.step(30)                           # a contact state
    y = G.get_state()[0]
    G.ip_assemble(y)
    rp, col, val = G.hessian_bsr()
    rhs = np.random.default_rng(4).normal(size=G.n_dof)
    for rtol in (1e-4, 1e-7):
        x, it, rr = G.pcg_solve(rhs, rtol=rtol)
        x = x.cpu().numpy()
        true = np.linalg.norm(rhs - bsr_matvec(rp, col, val, x)) / np.linalg.norm(rhs)
        log(f"mixed rtol {rtol}: {it} iterations, reported {rr:.3e}, true FP64 residual {true:.3e}")
        assert true <= rtol * (1 + 1e-9)
        assert abs(rr - true) <= 1e-3 * true + 1e-15
