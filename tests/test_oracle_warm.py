"""Pins of the FP64 reference of the learned initial guess's features and target.

* the closest point of a triangle is optimal against dense samples of the triangle
  and its distance equals the oracle's C++ point-triangle distance (an independent
  implementation);
* cube lowered to 2 mm above the slab, uniform velocity: bottom vertices see the slab
  at d = 2 dhat straight down, a static closest point and no driven body; every
  other vertex sees nothing in range; the velocity entries are v / 0.05 m/s;
* gripper with both fingers inside 4 dhat of the object, fingers at rest: vertices
  next to a finger see that finger's target velocity, |h tv / s| = 1;
* the training target of a free-fall step of an unconstrained body equals the
  gravity displacement h^2 g / s up to the Newton tolerance (no contact, no elastic
  force: every vertex moves by h v + h^2 g when the body stays undeformed).
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import ref, warm


def test_closest_point_is_optimal():
    rng = np.random.default_rng(0)
    uv = rng.uniform(size=(4000, 2))
    uv = uv[uv.sum(1) <= 1.0]
    for _ in range(60):
        a, b, c = rng.normal(size=(3, 3))
        p = rng.normal(size=3) * 1.5
        cp, w = warm.closest_point_triangle(p, a, b, c)
        assert abs(sum(w) - 1.0) < 1e-12 and min(w) >= -1e-12
        assert np.allclose(cp, w[0] * a + w[1] * b + w[2] * c, atol=1e-12)
        d = np.linalg.norm(p - cp)
        samples = a + uv[:, :1] * (b - a) + uv[:, 1:] * (c - a)
        assert d <= np.linalg.norm(samples - p, axis=1).min() + 1e-12
        assert d == pytest.approx(ref.dist_pt(np.concatenate([p, a, b, c]))[0], rel=1e-10, abs=1e-14)


def lowered_cube(dy=-0.003):
    sc = sg.cube_drop()
    sc.softs[0].pos0 = sc.softs[0].rest_pos + np.array([0.0, dy, 0.0])
    return sc


def test_cube_features_closed_form():
    sc = lowered_cube()
    R = ref.RefScene(sc)
    y, _, _, _ = R.get_state()
    nsv = R.n_soft_verts
    yd = np.zeros_like(y)
    vel = np.array([0.3, -1.0, 0.2])
    yd[:3 * nsv] = np.tile(vel, nsv)
    F = warm.features(sc, R, y, yd, np.zeros_like(y), 0)
    X = y[:3 * nsv].reshape(-1, 3)
    bottom = np.isclose(X[:, 1], X[:, 1].min())
    assert bottom.sum() == 25
    assert np.allclose(F[:, 0:3], vel / 0.05) and np.allclose(F[:, 3:6], vel / 0.05)
    assert np.allclose(F[bottom, 6], X[bottom, 1] / sc.params.dhat) and np.allclose(F[bottom, 6], 2.0)
    assert np.allclose(F[bottom, 7:10], [0.0, -1.0, 0.0])
    assert not F[bottom, 10:16].any()
    assert np.all(F[~bottom, 6] == 4.0) and not F[~bottom, 7:16].any()


def test_gripper_target_velocity_feature():
    from test_gpu_parity import gripper_contact_state
    sc = sg.gripper(0, r=12)
    R = ref.RefScene(sc)
    y, yd = gripper_contact_state(sc, R, squeeze=1.0, noise=0.0)
    nsv = R.n_soft_verts
    yd = yd.copy()
    yd[3 * nsv:] = 0.0                               # fingers at rest
    F = warm.features(sc, R, y, yd, yd, 0)
    near = F[:, 6] < 4.0
    assert near.sum() > 0
    assert np.allclose(np.linalg.norm(F[near, 13:16], axis=1), 1.0)
    assert np.allclose(np.abs(F[near, 13]), 1.0)     # the closing axis is x
    assert not F[~near, 13:16].any()


def test_free_fall_target():
    sc = sg.cube_drop()
    sc.affines = []                                  # nothing to touch
    R = ref.RefScene(sc)
    y0, yd0, _, _ = R.get_state()
    R.step(1)
    y1, _, _, _ = R.get_state()
    T = warm.warm_target(sc, y1, y0, yd0, R.n_soft_verts)
    h = sc.params.dt
    g = np.asarray(sc.params.gravity)
    # Newton stops once its step is below 1e-6 h = 1e-8 m, i.e. 2e-5 in units of s
    assert np.allclose(T, h * h * g / (h * 0.05), rtol=0, atol=1e-4)
