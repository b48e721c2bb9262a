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
