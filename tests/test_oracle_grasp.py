"""CPU pins of the grasp-evaluation pieces (Sec. IV-A controller, Sec. IV-B contact
force sensing, Sec. V procedure) in the oracle.

* phi (eq. 12): phi(0) = 1, phi(f*) = 0, zero beyond f*, strictly decreasing on
  [0, f*), and for k -> 0 the limit 1 - f/f* (expansion of both exponentials to first
  order) -- a dropped term, a swapped exponent or a wrong normalisation fails one.
* Contact forces: the force on a body is minus the derivative of the barrier energy
  under a rigid translation of that body, divided by h^2 (central differences of the
  oracle's barrier energy term; the definition written through the energy instead of
  the vertex gradients); the forces of all bodies sum to zero (each pair's distance is
  translation invariant); the settled cube's force on the slab equals its weight.
* Procedure: with the object resting on the ground the ground force is its weight; the
  controller closes the fingers (forces rise and stay below f*), the lift takes the
  object off the ground, and a trace row is written per step.
"""
import math

import numpy as np
import pytest

import scenegen as sg
from oracle import grasp, ref


def test_phi_endpoints_and_monotone():
    for k, fs in ((20.0, 0.5), (5.0, 1.0), (60.0, 0.2)):
        assert grasp.phi(0.0, k, fs) == pytest.approx(1.0, abs=1e-15)
        assert grasp.phi(fs, k, fs) == 0.0
        assert grasp.phi(2 * fs, k, fs) == 0.0
        assert grasp.phi(fs * (1 - 1e-12), k, fs) >= 0.0
        f = np.linspace(0.0, fs, 200, endpoint=False)
        v = np.array([grasp.phi(x, k, fs) for x in f])
        assert np.all(np.diff(v) < 0) and np.all(v > 0) and np.all(v <= 1.0)


def test_phi_small_k_limit_is_linear():
    fs = 0.5
    for f in (0.0, 0.1, 0.25, 0.4):
        assert grasp.phi(f, 1e-7, fs) == pytest.approx(1.0 - f / fs, abs=1e-6)


def test_phi_paper_constants():
    # k = 20 / N, f* = 0.5 N: half way to f* the gain is (e^-5 - e^-10) / (1 - e^-10)
    e5, e10 = 6.737946999085467e-03, 4.5399929762484854e-05
    assert grasp.phi(0.25, 20.0, 0.5) == pytest.approx((e5 - e10) / (1 - e10), rel=1e-12)


@pytest.fixture(scope="module")
def cube_contact():
    sc = sg.cube_drop()
    R = ref.RefScene(sc)
    R.step(4)                                 # the cube is in contact with the slab
    return sc, R


def _translate_body(R, sc, y, body, axis, eps):
    """y with soft body `body` (all its vertices) translated by eps along axis."""
    yy = y.copy()
    v0 = sum(len(b.rest_pos) for b in sc.softs[:body])
    n = len(sc.softs[body].rest_pos)
    yy[3 * v0 + axis:3 * (v0 + n):3] += eps
    return yy


def test_force_is_translation_derivative_of_barrier(cube_contact):
    sc, R = cube_contact
    y = R.get_state()[0]
    F = R.contact_forces(y)
    h2 = sc.params.dt ** 2
    assert np.linalg.norm(F[0]) > 0
    for axis in range(3):
        eps = 1e-8
        ep = R.ip_assemble(_translate_body(R, sc, y, 0, axis, eps), grad=False, hess=False)[0][4]
        em = R.ip_assemble(_translate_body(R, sc, y, 0, axis, -eps), grad=False, hess=False)[0][4]
        fd = -(ep - em) / (2 * eps) / h2
        assert abs(F[0][axis] - fd) <= 1e-5 * np.linalg.norm(F[0]) + 1e-12, (axis, F[0][axis], fd)


def test_forces_sum_to_zero(cube_contact):
    sc, R = cube_contact
    F = R.contact_forces(R.get_state()[0])
    scale = np.abs(F).max()
    assert scale > 0
    assert np.abs(F.sum(0)).max() <= 1e-10 * scale


def test_settled_cube_presses_slab_with_its_weight():
    sc = sg.cube_drop(steps=100)
    R = ref.RefScene(sc)
    R.step(100)
    F = R.contact_forces(R.get_state()[0])
    W = R.lumped_mass().sum() * 9.81
    # soft cube: body 0; fixed slab: body 1 (soft bodies first)
    assert F[1][1] == pytest.approx(-W, rel=1e-2)
    assert F[0][1] == pytest.approx(W, rel=1e-2)


def test_grasp_procedure_closes_and_lifts():
    sc = sg.grasp_scene(0, r=6)
    R = ref.RefScene(sc)
    res, tr = grasp.run(R, sc, f_star=0.5, max_close_steps=24, lift_steps=8, shake_steps=0, ground_body=3)
    assert res["n_fingers"] == 2 and tr.shape == (res["total_steps"], 4)
    close = tr[tr[:, 0] == 0]
    # before the fingers touch, the ground carries the whole weight (within the rounding
    # of the settled barrier)
    m = R.lumped_mass().sum()
    assert close[0, 1] == pytest.approx(m * 9.81, rel=0.05) or close[0, 1] == 0.0
    assert close[-1, 2] > 0 and close[-1, 3] > 0 and close[-1, 2] < 0.5 and close[-1, 3] < 0.5
    lift = tr[tr[:, 0] == 1]
    assert lift[-1, 1] == 0.0                 # off the ground
    assert res["success"] == 1
