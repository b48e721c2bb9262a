"""Pins of the oracle's per-element energies, gradients and projected Hessians.

Neo-Hookean (Sec. IV-D): zero energy and gradient at rest and under rigid motion,
small-strain limit equal to linear elasticity with the same Lame parameters,
central-difference gradient/Hessian, PSD after projection.  Orthogonality
(Sec. III eq. 2): zero energy and gradient on rotations.  Barrier pairs (eqs. 4-8,
with the edge-edge mollifier): central differences.  Friction (eqs. 9-10):
Coulomb limit mu*lambda when sliding, closed-form lambda, central differences, PSD.
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import ref


def rot(seed):
    return sg.uniform_rotation(np.random.default_rng(seed))


@pytest.fixture(scope="module")
def cube():
    s = sg.cube_drop()
    return s, ref.RefScene(s)


def tet_rest(s, e):
    b = s.softs[0]
    return b.rest_pos[b.tets[e]]


def test_tet_rest_and_rigid(cube):
    s, R = cube
    for e in (0, 7, 100):
        X = tet_rest(s, e)
        E, g, H = R.tet_energy(e, X.ravel())
        assert abs(E) < 1e-18 and np.abs(g).max() < 1e-14
        Q = rot(e)
        x = X @ Q.T + np.array([0.3, -0.2, 0.1])
        E, g, H = R.tet_energy(e, x.ravel())
        assert abs(E) < 1e-17 and np.abs(g).max() < 1e-13


def test_tet_small_strain_limit(cube):
    s, R = cube
    b = s.softs[0]
    mu = b.E / (2 * (1 + b.nu)); lam = b.E * b.nu / ((1 + b.nu) * (1 - 2 * b.nu))
    X = tet_rest(s, 3)
    V = np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1)) / 6
    G = np.random.default_rng(0).normal(size=(3, 3))
    eps = 1e-5
    E, _, _ = R.tet_energy(3, (X @ (np.eye(3) + eps * G).T).ravel())
    psi = E / (s.params.dt ** 2 * V) / eps ** 2
    S = 0.5 * (G + G.T)
    lin = mu * (S * S).sum() + 0.5 * lam * np.trace(G) ** 2
    assert abs(psi - lin) <= 1e-3 * lin


@pytest.mark.parametrize("seed", range(4))
def test_tet_fd_and_psd(cube, seed):
    s, R = cube
    X = tet_rest(s, 11)
    x = (X + np.random.default_rng(seed).normal(scale=3e-3, size=X.shape)).ravel()
    E, g, H = R.tet_energy(11, x, project=False)
    _, _, P = R.tet_energy(11, x, project=True)
    d = 1e-7
    gfd = np.zeros(12); Hfd = np.zeros((12, 12))
    for k in range(12):
        e = np.zeros(12); e[k] = d
        gfd[k] = (R.tet_energy(11, x + e, project=False)[0] - R.tet_energy(11, x - e, project=False)[0]) / (2 * d)
        Hfd[:, k] = (R.tet_energy(11, x + e, project=False)[1] - R.tet_energy(11, x - e, project=False)[1]) / (2 * d)
    assert np.abs(gfd - g).max() <= 1e-6 * np.abs(g).max()
    assert np.abs(Hfd - H).max() <= 1e-6 * np.abs(H).max()
    assert np.abs(P - P.T).max() <= 1e-14 * np.abs(P).max()
    assert np.linalg.eigvalsh(P).min() >= -1e-12 * np.abs(P).max()
    # translation is in the null space of the projected Hessian
    t = np.tile([1.0, 0.0, 0.0], 4)
    assert np.abs(P @ t).max() <= 1e-10 * np.abs(P).max()


def test_tet_inverted_is_infinite(cube):
    s, R = cube
    X = tet_rest(s, 0).copy()
    X[[1, 2]] = X[[2, 1]]
    assert R.tet_energy(0, X.ravel())[0] == float("inf")


def free_box_scene():
    v, t = sg.box_surface((0.0, 0.0, 0.0), (0.05, 0.02, 0.03), 2)
    p = sg.Params(dt=0.01, gravity=(0.0, 0.0, 0.0))
    return sg.Scene("free_box", p, [], [sg.AffineBody(v, t, stiffness=1e5, mode=sg.MODE_FREE)], 1)


def test_orthogonality_rotation_invariant():
    s = free_box_scene()
    R = ref.RefScene(s)
    y, yd, _, _ = R.get_state()
    for seed in range(3):
        Q = rot(seed)
        y1 = y.copy(); y1[3:] = Q.ravel()          # rows of A = rows of Q
        terms, g = R.ip_assemble(y1, mask=1 << 2)
        assert abs(terms[2]) < 1e-20 and np.abs(g).max() < 1e-14
    y1 = y.copy(); y1[3:] = (1.01 * rot(5)).ravel()
    terms, g = R.ip_assemble(y1, mask=1 << 2)
    assert terms[2] > 0
    # central differences of the orthogonality energy
    d = 1e-7
    for k in (3, 7, 11):
        e = np.zeros_like(y1); e[k] = d
        fd = (R.ip_assemble(y1 + e, grad=False, hess=False)[0][2] - R.ip_assemble(y1 - e, grad=False, hess=False)[0][2]) / (2 * d)
        assert abs(fd - g[k]) <= 1e-6 * np.abs(g).max()


def _fd_pair(R, kind, x, rl):
    E, g, H = R.pair_energy(kind, x, rl, project=False)
    d = 1e-9
    gfd = np.zeros(12); Hfd = np.zeros((12, 12))
    for k in range(12):
        e = np.zeros(12); e[k] = d
        Ep, gp, _ = R.pair_energy(kind, x + e, rl, project=False)
        Em, gm, _ = R.pair_energy(kind, x - e, rl, project=False)
        gfd[k] = (Ep - Em) / (2 * d)
        Hfd[:, k] = (gp - gm) / (2 * d)
    return E, g, H, gfd, Hfd


@pytest.mark.parametrize("case", ["pt_face", "pt_edge", "ee_cross", "ee_mollified"])
def test_pair_energy_fd(cube, case):
    s, R = cube
    rng = np.random.default_rng(hash(case) % 1000)
    if case == "pt_face":
        t = np.array([[0, 0, 0], [0.01, 0, 0], [0, 0, 0.01]], float) + rng.normal(scale=1e-4, size=(3, 3))
        p = np.array([0.003, 4e-4, 0.003])
        x = np.concatenate([p, t.ravel()]); kind = 0; rl = (1.0, 1.0)
    elif case == "pt_edge":
        t = np.array([[0, 0, 0], [0.01, 0, 0], [0, 0, 0.01]], float)
        p = np.array([0.005, 3e-4, -3e-4])
        x = np.concatenate([p, t.ravel()]); kind = 0; rl = (1.0, 1.0)
    elif case == "ee_cross":
        x = np.array([-0.01, 0, 0, 0.01, 0, 0, 0.001, -0.01, 5e-4, -0.001, 0.01, 5e-4]); kind = 1
        rl = (4e-4, 4e-4)
    else:
        x = np.array([-0.01, 0, 0, 0.01, 0, 0, -0.01, 1e-5, 5e-4, 0.01, -1e-5, 5e-4]); kind = 1
        rl = (4e-4, 4e-4)   # eps = 1.6e-10 > |ea x eb|^2
    E, g, H, gfd, Hfd = _fd_pair(R, kind, x, rl)
    assert E > 0
    assert np.abs(gfd - g).max() <= 1e-5 * np.abs(g).max()
    assert np.abs(Hfd - H).max() <= 1e-4 * np.abs(H).max()
    _, _, P = R.pair_energy(kind, x, rl, project=True)
    assert np.linalg.eigvalsh(P).min() >= -1e-12 * np.abs(P).max()


def test_pair_typed_matches_closest_and_tie_closed_form(cube):
    """The typed pair evaluation (test use: the other side of a feature tie).  Away from
    a tie the closest type gives the untyped result bitwise.  A point at height d above
    the midpoint of a triangle edge has the face and that edge at the same distance:
    energies and gradients agree, and the point's unprojected Hessian blocks differ by
    exactly kappa b'(d)/d m m^T, m the in-plane normal of the edge (the distance to the
    plane is linear in the point; the distance to a line has Hessian m m^T / d), with
    b'(d) = -2 (d - dhat) log(d / dhat) - (d - dhat)^2 / d of the log barrier (eq. 5)."""
    s, R = cube
    kappa = R.get_state()[2]
    dhat = s.params.dhat
    t = np.array([[0, 0, 0], [0.01, 0, 0], [0, 0, 0.01]], float)
    x = np.concatenate([[0.003, 4e-4, 0.002], t.ravel()])
    d, ty = ref.dist_pt(x)
    assert ty == 6
    e0, g0, H0 = R.pair_energy(0, x, project=False)
    e1, g1, H1 = R.pair_energy(0, x, project=False, ftype=ty)
    assert e0 == e1 and np.array_equal(g0, g1) and np.array_equal(H0, H1)
    for d in (2e-4, 5e-4, 9e-4):
        x = np.concatenate([[0.005, d, 0.0], t.ravel()])   # above the midpoint of edge t0 t1 (type 3)
        ef, gf, Hf = R.pair_energy(0, x, project=False, ftype=6)
        ee, ge, He = R.pair_energy(0, x, project=False, ftype=3)
        assert ef > 0 and abs(ee - ef) <= 1e-14 * ef
        assert np.abs(ge - gf).max() <= 1e-12 * np.abs(gf).max()
        bp = -2.0 * (d - dhat) * np.log(d / dhat) - (d - dhat) ** 2 / d
        m = np.array([0.0, 0.0, 1.0])
        want = kappa * bp / d * np.outer(m, m)
        assert np.abs((He - Hf)[:3, :3] - want).max() <= 1e-9 * np.abs(want).max()
        assert bp < 0


def contact_tet_scene(mu=0.5):
    v0 = np.array([0.02, 5e-4, -0.01])
    v = np.array([v0, v0 + [0.02, 0.01, 0], v0 + [0, 0.02, 0], v0 + [0, 0.01, 0.02]])
    sv, st = sg.box_surface((0.0, -0.01, 0.0), (0.05, 0.01, 0.05), 1)
    p = sg.Params(dt=0.01, dhat=1e-3, mu=mu, eps_v=1e-3)
    return sg.Scene("contact_tet", p, [sg.SoftBody(v, np.array([[0, 1, 2, 3]], np.int32), 1e5, 0.4, 1000.0)],
                    [sg.AffineBody(sv, st, mode=sg.MODE_FIXED)], 1)


def test_friction_coulomb_and_lambda():
    s = contact_tet_scene()
    R = ref.RefScene(s)
    y, yd, kappa, _ = R.get_state()
    ids, vals = R.friction_table()
    assert len(ids) == 1 and ids[0, 0] == 0
    dh = s.params.dhat; d = 5e-4
    bp = -2 * (d - dh) * np.log(d / dh) - (d - dh) ** 2 / d
    lam = vals[0, 0]
    assert abs(lam - kappa * abs(bp)) <= 1e-12 * lam
    assert np.allclose(vals[0, 1:4], [0, 1, 0], atol=1e-12)
    # sliding: tangential displacement larger than eps_v h -> force magnitude mu lambda
    y1 = y.copy(); y1[0:12:3] += 3e-4
    terms, g = R.ip_assemble(y1, mask=1 << 5)
    assert abs(g[0] - s.params.mu * lam) <= 1e-12 * lam
    assert np.abs(g[1:3]).max() <= 1e-12 * lam and np.abs(g[3:]).max() == 0.0
    assert abs(terms[5] - s.params.mu * lam * 3e-4) <= 1e-12 * terms[5]
    # static zone: closed form mu lambda f1(y)/y u
    ys = s.params.eps_v * s.params.dt
    u = 0.3 * ys
    y2 = y.copy(); y2[0:12:3] += u
    terms, g = R.ip_assemble(y2, mask=1 << 5)
    f1 = 2 * u / ys - u * u / ys ** 2
    assert abs(g[0] - s.params.mu * lam * f1) <= 1e-12 * lam
    f0 = -u ** 3 / (3 * ys ** 2) + u ** 2 / ys + ys / 3
    assert abs(terms[5] - s.params.mu * lam * f0) <= 1e-12 * s.params.mu * lam * ys


@pytest.mark.parametrize("disp", [2e-6, 3e-5])
def test_friction_fd_and_psd(disp):
    s = contact_tet_scene()
    R = ref.RefScene(s)
    y, _, _, _ = R.get_state()
    y1 = y.copy(); y1[0] += disp; y1[2] -= 0.5 * disp; y1[1] += 1e-5
    terms, g = R.ip_assemble(y1, mask=1 << 5)
    H = np.stack([R.hessian_matvec(e) for e in np.eye(R.n_dof)], 1)
    d = 1e-9
    for k in range(3):
        e = np.zeros_like(y1); e[k] = d
        fp = R.ip_assemble(y1 + e, grad=False, hess=False)[0][5]
        fm = R.ip_assemble(y1 - e, grad=False, hess=False)[0][5]
        assert abs((fp - fm) / (2 * d) - g[k]) <= 1e-5 * np.abs(g).max()
    # Hessian of the friction term alone is symmetric PSD
    R.ip_assemble(y1, mask=1 << 5)
    H = np.stack([R.hessian_matvec(e) for e in np.eye(R.n_dof)], 1)
    assert np.abs(H - H.T).max() <= 1e-12 * np.abs(H).max()
    assert np.linalg.eigvalsh(H).min() >= -1e-12 * np.abs(H).max()
    # FD of the friction gradient
    for k in range(3):
        e = np.zeros_like(y1); e[k] = d
        gp = R.ip_assemble(y1 + e, hess=False, mask=1 << 5)[1]
        gm = R.ip_assemble(y1 - e, hess=False, mask=1 << 5)[1]
        assert np.abs((gp - gm) / (2 * d) - H[:, k]).max() <= 1e-5 * np.abs(H).max()
