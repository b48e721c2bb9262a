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
  force: every vertex moves by h v + h^2 g when the body stays undeformed);
* the per-body fit of a correction field: an affine field is its own affine fit and
  its mean is the field at the mass centre; a constant field is unchanged by every
  mode; the residual of the affine fit of a random field is mass-orthogonal to
  1 and to x - xbar on every body (the normal equations of the weighted least
  squares), and the fit of each body ignores the other bodies' values.
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


def two_bodies():
    """The soft cube and a shifted, sheared copy of it: two soft bodies in one scene."""
    sc = sg.cube_drop()
    a = sc.softs[0]
    b = sg.SoftBody(a.rest_pos @ np.array([[1.0, 0.2, 0], [0, 1.0, 0], [0, 0.1, 0.9]]) + [0.3, 0.05, -0.1],
                    a.tets.copy(), a.E, a.nu, a.rho)
    return sg.Scene("two_cubes", sc.params, [a, b], sc.affines, 1)


def test_fit_correction_pins():
    sc = two_bodies()
    R = ref.RefScene(sc)
    m = R.lumped_mass()
    y = R.get_state()[0]
    n = R.n_soft_verts
    rng = np.random.default_rng(5)
    y = y.copy()
    y[:3 * n] += rng.normal(scale=2e-3, size=3 * n)
    x = y[:3 * n].reshape(-1, 3)
    n0 = len(sc.softs[0].rest_pos)
    parts = [slice(0, n0), slice(n0, n)]
    # affine per body
    aff = np.zeros((n, 3))
    maps = []
    for sl in parts:
        t, B = rng.normal(size=3), rng.normal(size=(3, 3))
        aff[sl] = t + x[sl] @ B.T
        maps.append((t, B))
    f1 = warm.fit_correction(sc, m, y, aff, 1)
    assert np.abs(f1 - aff).max() <= 1e-12 * np.abs(aff).max()
    f2 = warm.fit_correction(sc, m, y, aff, 2)
    for sl, (t, B) in zip(parts, maps):
        xc = m[sl] @ x[sl] / m[sl].sum()
        assert np.abs(f2[sl] - (t + B @ xc)).max() <= 1e-12 * np.abs(aff).max()
    const = np.tile([0.3, -1.2, 0.7], (n, 1))
    for mode in (0, 1, 2):
        assert np.abs(warm.fit_correction(sc, m, y, const, mode) - const).max() <= 1e-14
    c = rng.normal(size=(n, 3))
    f = warm.fit_correction(sc, m, y, c, 1)
    for sl in parts:
        r, w = c[sl] - f[sl], m[sl]
        X = x[sl] - w @ x[sl] / w.sum()
        assert np.abs(w @ r).max() <= 1e-12 * np.abs(w[:, None] * c[sl]).sum()
        assert np.abs((X * w[:, None]).T @ r).max() <= 1e-12 * np.abs(X).max() * np.abs(w[:, None] * c[sl]).sum()
    c2 = c.copy()
    c2[parts[1]] += 5.0
    f_2 = warm.fit_correction(sc, m, y, c2, 1)
    assert np.array_equal(f_2[parts[0]], f[parts[0]])

