"""Pins of the oracle's affine-body terms.

* Predictor and inertia of an affine body (Sec. III eqs. 2-3): with the rest shape
  measured from the centre of mass, gravity acts on q as (g, 0, 0, 0), so a free body
  translating in flight has p^{t+1} = p^t + h pdot^t + h^2 g and keeps A = I.
* Linear momentum of a free soft body and a free affine body colliding in flight
  (both potentials and the contact terms are translation invariant; the affine
  body's momentum is m pdot because x0 is centred).
* Chain rule into affine DOFs (Sec. III eqs. 6-8): central differences of the barrier
  and friction energies with respect to each of the 12 q entries of a free body equal
  the gradient; the barrier Hessian in q equals J^T P J with J built here from
  x = A x0 + p and P the projected x-space pair Hessian; the friction term is convex,
  so central differences of its gradient equal its Hessian.
* Kinematic penalty (Sec. IV-C-1, eq. 13 with a zero multiplier): energy
  kappa_A/2 |q - q~|^2 with the target moved at its velocity until the stop time,
  gradient kappa_A (q - q~), Hessian kappa_A I, and the closed-form minimiser of one
  step, p = (m p^ + kappa_A p~) / (m + kappa_A).
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import ref


def tilted_box(center, half, angles):
    """Surface (one quad per face) of a box rotated about z, then x, then moved."""
    v, t = sg.box_surface((0.0, 0.0, 0.0), half, 1)
    cz, sz = np.cos(angles[0]), np.sin(angles[0])
    cx, sx = np.cos(angles[1]), np.sin(angles[1])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    return v @ (Rx @ Rz).T + center, t


def corner_on_slab(gap, dt=0.01, mu=0.5):
    """A free affine box resting on one corner `gap` above the interior of a fixed
    slab's top face (far from the face's diagonal x = z and its border), no gravity:
    exactly one contact pair (the corner against one slab triangle) is active."""
    half = (0.02, 0.015, 0.01)
    v, t = tilted_box((0.0, 0.0, 0.0), half, (0.5, 0.6))
    low = np.argmin(v[:, 1])
    v = v + (np.array([0.05, gap, -0.1]) - v[low])
    slab_v, slab_t = sg.box_surface((0.0, -0.025, 0.0), (0.25, 0.025, 0.25), 1)
    p = sg.Params(dt=dt, dhat=1e-3, mu=mu, eps_v=1e-3, gravity=(0.0, 0.0, 0.0))
    box = sg.AffineBody(v, t, rho=800.0, stiffness=1e8, mode=sg.MODE_FREE)
    slab = sg.AffineBody(slab_v, slab_t, mode=sg.MODE_FIXED)
    center = v.mean(axis=0)             # the box's centre of mass (8 symmetric corners)
    return sg.Scene("corner", p, [], [box, slab], 1), v, low, center


def jacobian(x0):
    """dx/dq of x = A x0 + p for q = (p, a1, a2, a3), a_r the rows of A (eq. 2)."""
    J = np.zeros((3, 12))
    for r in range(3):
        J[r, r] = 1.0
        J[r, 3 + 3 * r:6 + 3 * r] = x0
    return J


def active_pairs(R, y):
    xs = R.surface_positions(y)
    tris, edges, _ = R.surface()
    pt, ee = R.candidates(xs)
    act = []
    for v, t in pt:
        d, _ = ref.dist_pt(np.concatenate([xs[v], xs[tris[t]].ravel()]))
        if d < R.params.dhat:
            act.append((0, v, t, d))
    for a, b in ee:
        d, _ = ref.dist_ee(np.concatenate([xs[edges[a]].ravel(), xs[edges[b]].ravel()]))
        if d < R.params.dhat:
            act.append((1, a, b, d))
    return act, xs, tris


def fd_grad(R, y, term, idx, delta):
    out = np.zeros(len(idx))
    for n, k in enumerate(idx):
        e = np.zeros_like(y); e[k] = delta[n]
        Ep = R.ip_assemble(y + e, grad=False, hess=False)[0][term]
        Em = R.ip_assemble(y - e, grad=False, hess=False)[0][term]
        out[n] = (Ep - Em) / (2 * delta[n])
    return out


def q_steps(x0):
    """Central-difference steps for q: 1e-8 m on p, 1e-8 m / |x0| on the rows of A."""
    s = 1e-8 / np.abs(x0).max()
    return np.array([1e-8] * 3 + [s] * 9)


def test_affine_free_fall_closed_form():
    v, t = sg.box_surface((0.01, 0.3, -0.02), (0.03, 0.02, 0.025), 2)
    qd = np.zeros(12); qd[:3] = [0.4, 1.5, -0.2]
    p = sg.Params(dt=0.01)
    s = sg.Scene("affine_fall", p, [], [sg.AffineBody(v, t, rho=600.0, qdot0=qd, mode=sg.MODE_FREE)], 4)
    R = ref.RefScene(s)
    y, yd, _, _ = R.get_state()
    assert np.allclose(y, [0.01, 0.3, -0.02, 1, 0, 0, 0, 1, 0, 0, 0, 1], atol=1e-15)
    h, g = p.dt, np.array(p.gravity)
    pos, vel = y[:3].copy(), qd[:3].copy()
    for _ in range(4):
        R.step(1)
        pos = pos + h * vel + h * h * g
        vel = vel + h * g
        y, yd, _, _ = R.get_state()
        assert np.abs(y[:3] - pos).max() <= 1e-12
        assert np.abs(yd[:3] - vel).max() <= 1e-10
        assert np.abs(y[3:] - np.eye(3).ravel()).max() <= 1e-14
        assert np.abs(yd[3:]).max() <= 1e-12


def test_momentum_soft_and_affine_collide_in_flight():
    s = sg.cube_drop()
    soft = s.softs[0]
    lift = np.array([0.0, 1.0, 0.0])
    bv, bt = sg.box_surface((0.0171, 1.0 + 0.005 + 0.1 + 0.0016 + 0.02, -0.0093), (0.03, 0.02, 0.03), 2)
    qd = np.zeros(12); qd[:3] = [0.05, -0.4, 0.02]
    rho_b = 500.0
    box = sg.AffineBody(bv, bt, rho=rho_b, stiffness=1e8, mode=sg.MODE_FREE, qdot0=qd)
    sc = sg.Scene("collide", s.params, [sg.SoftBody(soft.rest_pos + lift, soft.tets, soft.E, soft.nu, soft.rho)],
                  [box], 4)
    R = ref.RefScene(sc)
    m = R.lumped_mass()
    mb = rho_b * 0.06 * 0.04 * 0.06                 # box mass from its size
    M = m.sum() + mb
    ns = 3 * R.n_soft_verts

    def momentum():
        _, yd, _, _ = R.get_state()
        return (m[:, None] * yd[:ns].reshape(-1, 3)).sum(0) + mb * yd[ns:ns + 3]

    P = momentum()
    h, g = sc.params.dt, np.array(sc.params.gravity)
    touched = 0
    for k in range(4):
        st = R.step(1)[0]
        touched += st["n_pt_active"] + st["n_ee_active"]
        P = P + h * M * g
        # Newton stops at max |dx| <= 1e-6 h; PCG leaves a relative 1e-4 residual
        assert np.abs(momentum() - P).max() <= 2e-6 * M, (k, momentum() - P)
    assert touched > 0                               # the bodies did collide


def test_chain_rule_barrier_and_friction_single_corner():
    sc, v, low, center = corner_on_slab(0.5e-3)
    R = ref.RefScene(sc)
    y0, _, kappa, _ = R.get_state()
    assert np.allclose(y0[:3], center, atol=1e-15)
    act, xs, tris = active_pairs(R, y0)
    assert len(act) == 1 and act[0][0] == 0 and act[0][1] == low
    x0 = v[low] - center
    J = jacobian(x0)
    # barrier: FD in q, and the q Hessian J^T P J with the projected x-space Hessian
    A = np.eye(3) + 1e-3 * np.array([[0.3, -0.2, 0.1], [0.2, 0.1, -0.4], [-0.1, 0.3, 0.2]])
    y = y0.copy(); y[3:] = A.ravel(); y[:3] += [2e-5, 1e-4, -3e-5]
    act, xs, tris = active_pairs(R, y)
    assert len(act) == 1
    _, vtx, tri, d = act[0]
    assert 0 < d < 1e-3
    terms, g = R.ip_assemble(y, mask=1 << 4)
    gfd = fd_grad(R, y, 4, range(12), q_steps(x0))
    assert np.abs(gfd - g).max() <= 1e-6 * np.abs(g).max()
    Hq = np.stack([R.hessian_matvec(e) for e in np.eye(12)], 1)
    x12 = np.concatenate([xs[vtx], xs[tris[tri]].ravel()])
    E, g12, P = R.pair_energy(0, x12, project=True)
    assert abs(E - terms[4]) <= 1e-12 * E
    assert np.abs(J.T @ g12[:3] - g).max() <= 1e-12 * np.abs(g).max()
    Hx = J.T @ P[:3, :3] @ J
    assert np.abs(Hq - Hx).max() <= 1e-10 * np.abs(Hx).max()
    # friction (lagged at y0): FD of energy and of gradient in q, sliding and static
    for disp in (3e-6, 2e-5):
        y = y0.copy(); y[0] += disp; y[2] -= 0.5 * disp
        terms, g = R.ip_assemble(y, mask=1 << 5)
        assert terms[5] > 0
        gfd = fd_grad(R, y, 5, range(12), q_steps(x0))
        assert np.abs(gfd - g).max() <= 1e-6 * np.abs(g).max()
        Hq = np.stack([R.hessian_matvec(e) for e in np.eye(12)], 1)
        Hfd = np.zeros((12, 12))
        for k, dk in enumerate(q_steps(x0)):
            e = np.zeros(12); e[k] = dk
            gp = R.ip_assemble(y + e, hess=False, mask=1 << 5)[1]
            gm = R.ip_assemble(y - e, hess=False, mask=1 << 5)[1]
            Hfd[:, k] = (gp - gm) / (2 * dk)
        assert np.abs(Hfd - Hq).max() <= 1e-5 * np.abs(Hq).max()


@pytest.fixture(scope="module")
def box_on_cube_contact():
    s = sg.box_on_cube()
    R = ref.RefScene(s)
    for _ in range(12):
        st = R.step(1)[0]
        y = R.get_state()[0]
        ns = 3 * R.n_soft_verts
        act, _, _ = active_pairs(R, y)
        tris, edges, vb = R.surface()
        box_pairs = 0
        for kind, a, b, _ in act:
            ids = [a] if kind == 0 else list(edges[a])
            other = tris[b] if kind == 0 else edges[b]
            bodies = {vb[i] for i in list(ids) + list(other)}
            box_pairs += 1 in bodies
        if box_pairs >= 4:
            return s, R, y, ns
    pytest.fail("the box never touched the cube")


def test_chain_rule_fd_box_on_cube(box_on_cube_contact):
    s, R, y, ns = box_on_cube_contact
    x0max = 0.03 * np.sqrt(3)
    steps = np.array([1e-8] * 3 + [1e-8 / x0max] * 9)
    qi = list(range(ns, ns + 12))
    for term in (4, 5):
        yq = y.copy()
        if term == 5:                  # slide the box against the lagged contacts
            yq[ns] += 4e-6; yq[ns + 2] -= 2e-6
        terms, g = R.ip_assemble(yq, mask=1 << term)
        assert terms[term] > 0
        gfd = fd_grad(R, yq, term, qi, steps)
        gq = g[ns:ns + 12]
        assert np.abs(gfd - gq).max() <= 1e-5 * np.abs(gq).max(), (term, gfd, gq)


def driven_box(kappa_A, vel, stop, dt=0.01):
    v, t = sg.box_surface((0.0, 0.0, 0.0), (0.02, 0.02, 0.02), 1)
    p = sg.Params(dt=dt)
    qd = np.zeros(12)
    body = sg.AffineBody(v, t, rho=1000.0, mode=sg.MODE_DRIVEN, kappa_A=kappa_A, qdot0=qd,
                         target_vel=np.asarray(vel, float), target_stop=stop)
    return sg.Scene("driven", p, [], [body], 6), 1000.0 * 0.04 ** 3


def test_kinematic_penalty_terms():
    kA, vel, stop = 3e3, np.array([0.1, -0.05, 0.02]), 0.025
    sc, m = driven_box(kA, vel, stop)
    R = ref.RefScene(sc)
    y0, yd0, _, _ = R.get_state()
    rng = np.random.default_rng(4)
    for step in (0, 1, 2, 5):          # target time (step + 1) h: 0.01 .. 0.06 (held past 0.025)
        R.set_state(y0, yd0, 0.0, step)
        qt = y0.copy()
        qt[:3] += min((step + 1) * sc.params.dt, stop) * vel
        y = y0 + rng.normal(scale=1e-3, size=12)
        terms, g = R.ip_assemble(y, mask=1 << 3)
        assert abs(terms[3] - 0.5 * kA * ((y - qt) ** 2).sum()) <= 1e-12 * terms[3]
        assert np.abs(g - kA * (y - qt)).max() <= 1e-12 * np.abs(g).max()
        H = np.stack([R.hessian_matvec(e) for e in np.eye(12)], 1)
        assert np.abs(H - kA * np.eye(12)).max() <= 1e-12 * kA


def test_kinematic_penalty_step_closed_form():
    kA, vel, stop = 3e3, np.array([0.1, -0.05, 0.02]), 0.025
    sc, m = driven_box(kA, vel, stop)
    R = ref.RefScene(sc)
    y, _, _, _ = R.get_state()
    h, g = sc.params.dt, np.array(sc.params.gravity)
    p0 = y[:3].copy()
    pos, v = p0.copy(), np.zeros(3)
    for n in range(6):
        R.step(1)
        phat = pos + h * v + h * h * g
        ptil = p0 + min((n + 1) * h, stop) * vel
        new = (m * phat + kA * ptil) / (m + kA)
        v = (new - pos) / h
        pos = new
        yn, ydn, _, _ = R.get_state()
        assert np.abs(yn[:3] - pos).max() <= 1e-12, n
        assert np.abs(yn[3:] - np.eye(3).ravel()).max() <= 1e-14
        assert np.abs(ydn[:3] - v).max() <= 1e-9
