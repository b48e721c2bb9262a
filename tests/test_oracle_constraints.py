"""CPU pins of the constraint energies of Sec. IV-C in the oracle.

* Springs (Sec. IV-C-3, k |x - x_target|^2 per vertex): a free affine box under gravity
  hung from springs at all its surface vertices (targets at the rest positions, equal
  k) settles with a rigid sag m g / (2 k N), N springs; gradient of the constraint term
  through the affine vertex map against central differences.
* Augmented Lagrangian of the kinematic energy (eq. 13): a driven box held at its rest
  pose under gravity.  Penalty only, the hold sags by m h^2 g / kappa_A in the
  translation (the kinematic gradient balances the inertia term's -m h^2 g); with
  multiplier updates the residual falls below the tolerance and sqrt(m) lambda_A of
  the translation tends to m h^2 |g| upwards (the constraint force in
  incremental-potential units).
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import ref


def test_springs_hold_box_with_rigid_sag():
    sc = sg.held_box(mode=sg.MODE_FREE, steps=60)
    R = ref.RefScene(sc)
    y0 = R.get_state()[0]
    xs0 = R.surface_positions(y0)
    n = len(xs0)
    k = 200.0
    R.set_springs(np.arange(n), np.full(n, k), xs0)
    R.step(60)
    y = R.get_state()[0]
    xs = R.surface_positions(y)
    sag = xs - xs0
    mass = sc.affines[0].rho * 0.04 ** 3
    expect = mass * 9.81 / (2 * k * n)
    assert np.abs(sag[:, 0]).max() < 1e-3 * expect and np.abs(sag[:, 2]).max() < 1e-3 * expect
    assert sag[:, 1] == pytest.approx(-expect, rel=2e-3)


def test_spring_gradient_matches_differences():
    sc = sg.held_box(mode=sg.MODE_FREE)
    R = ref.RefScene(sc)
    y = R.get_state()[0]
    xs0 = R.surface_positions(y)
    rng = np.random.default_rng(3)
    sv = np.array([0, 5, 11, 17])
    R.set_springs(sv, rng.uniform(50, 300, len(sv)), xs0[sv] + rng.normal(scale=0.003, size=(len(sv), 3)))
    yy = y + rng.normal(scale=1e-3, size=y.shape)
    _, g = R.ip_assemble(yy, hess=False, mask=1 << 3)
    for i in range(len(y)):
        e = np.zeros(len(y)); e[i] = 1e-6
        fd = (R.ip_assemble(yy + e, grad=False, hess=False)[0][3] - R.ip_assemble(yy - e, grad=False, hess=False)[0][3]) / 2e-6
        assert abs(g[i] - fd) <= 1e-6 * np.abs(g).max(), i


def test_kinematic_penalty_sag_and_multiplier():
    kA = 1e3
    sc = sg.held_box(kappa_A=kA, steps=5)
    h = sc.params.dt
    mass = sc.affines[0].rho * 0.04 ** 3
    R = ref.RefScene(sc)
    R.step(5)
    y = R.get_state()[0]
    q0 = ref.RefScene(sc).get_state()[0]
    sag = y[1] - q0[1]
    # held still: the inertia gradient at the hold is -m h^2 g, balanced by kappa_A sag
    # (to the accuracy of the Newton solve: PCG stops at 1e-4 of the residual)
    assert sag == pytest.approx(-mass * h * h * 9.81 / kA, rel=2e-3)
    R2 = ref.RefScene(sc)
    tol = 1e-3 * abs(sag)                     # above the Newton solve's own noise
    R2.kinematic_al(tol, 12)
    st = R2.step(5)
    y2 = R2.get_state()[0]
    assert abs(y2[1] - q0[1]) <= 1e-3 * abs(sag)   # the multiplier takes the load off the penalty
    lam = R2.kinematic_al(tol, 12)
    assert np.sqrt(mass) * lam[0][1] == pytest.approx(mass * h * h * 9.81, rel=2e-3)
    assert 1 <= sum(s["al_updates"] for s in st) <= 10


# ---------------------------------------------------------------- prismatic joint (Sec. IV-C-2)

def _slider(kappa=1e4):
    sc = sg.slider_scene()
    R = ref.RefScene(sc)
    R.set_prismatic_joints([[1, 0]], [[1.0, 0.0, 0.0]], [kappa])
    return sc, R


def test_joint_energy_closed_forms():
    kappa = 1e4
    sc, R = _slider(kappa)
    y0 = R.get_state()[0]                       # DOFs: the slider's q (the rail is fixed)
    assert len(y0) == 12
    E = lambda y: R.ip_assemble(y, grad=False, hess=False)[0][3]
    assert E(y0) == 0.0
    y = y0.copy(); y[0] += 0.013                 # along the axis: free
    assert abs(E(y)) <= 1e-20
    d = np.array([0.002, -0.003, 0.0015])
    y = y0.copy(); y[:3] += d                    # kappa |d_perp|^2
    assert E(y) == pytest.approx(kappa * (d[1] ** 2 + d[2] ** 2), rel=1e-12)
    th = 0.01                                    # relative rotation about z: kappa 4 (1 - cos th)
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    y = y0.copy(); y[3:12] = Rz.ravel()
    assert E(y) == pytest.approx(kappa * 4 * (1 - np.cos(th)), rel=1e-9)


def test_joint_gradient_matches_differences():
    sc, R = _slider(1e4)
    rng = np.random.default_rng(5)
    y = R.get_state()[0] + rng.normal(scale=2e-3, size=12)
    _, g = R.ip_assemble(y, hess=False, mask=1 << 3)
    for i in range(12):
        e = np.zeros(12); e[i] = 1e-7
        fd = (R.ip_assemble(y + e, grad=False, hess=False)[0][3] - R.ip_assemble(y - e, grad=False, hess=False)[0][3]) / 2e-7
        assert abs(g[i] - fd) <= 1e-6 * np.abs(g).max(), i


def test_joint_slides_freely_and_holds_perpendicular():
    kappa = 10.0       # soft enough that the sag is well above the Newton tolerance
    sc, R = _slider(kappa)
    y0 = R.get_state()[0]
    st = R.step(10)
    y = R.get_state()[0]
    h = sc.params.dt
    m = sc.affines[1].rho * 0.04 ** 3
    assert y[0] - y0[0] == pytest.approx(0.1 * 10 * h, rel=1e-6)       # constant axial velocity
    # perpendicular: the joint's 2 kappa dy balances the inertia term's m h^2 g
    assert y[1] - y0[1] == pytest.approx(-m * h * h * 9.81 / (2 * kappa), rel=2e-2)
    # the sagged gap r tilts A1 d towards r only slowly (|r x A1 d|^2 couples them)
    assert abs(y[2] - y0[2]) <= 1e-12 and np.abs(y[3:] - y0[3:]).max() <= 1e-6
