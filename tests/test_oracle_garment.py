"""Pins of the oracle's garment (Baraff-Witkin membrane, Sec. IV-D) against what the
definition fixes (test infrastructure for the library's garment kernels):

* mass: the lumped masses sum to rho times the sheet's area;
* the flat sheet at rest and under any rigid motion has zero elastic energy and
  gradient (|w_u| = |w_v| = 1, w_u . w_v = 0 are invariant);
* a uniform stretch by s along u gives h^2 area k_s/2 (s - 1)^2 (the v column keeps
  unit length, no shear); a uniform shear x += g z gives
  h^2 area (k_s/2 (sqrt(1 + g^2) - 1)^2 + k_sh/2 g^2) with k_sh = E / (2 (1 + nu));
* the gradient matches central differences of the energy at a random deformation;
* the projected Hessian is symmetric PSD, and under a pure stretch (s > 1 along u and
  v, no shear: every part convex there) it equals the central-difference Hessian;
* dropped onto the cone, the sheet stays intersection-free after every step (exact
  check) and falls rigidly by h^2 g in its first, contact-free step.
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import ref


@pytest.fixture(scope="module")
def sheet():
    sc = sg.garment_on_cone(n=4, side=0.2)
    return sc, ref.RefScene(sc)


def elastic(R, y):
    t, g = R.ip_assemble(y, hess=False, mask=1 << 1)
    return t[1], g


def test_mass_and_rest(sheet):
    sc, R = sheet
    assert R.lumped_mass().sum() == pytest.approx(sc.softs[0].rho * 0.2 ** 2, rel=1e-14)
    y = R.get_state()[0].copy()
    e, g = elastic(R, y)
    assert abs(e) <= 1e-30 and np.abs(g).max() <= 1e-18
    rng = np.random.default_rng(0)
    Q = sg.uniform_rotation(rng)
    n = R.n_soft_verts
    x = y[:3 * n].reshape(-1, 3) @ Q.T + rng.normal(size=3)
    y[:3 * n] = x.ravel()
    e, g = elastic(R, y)
    assert abs(e) <= 1e-25 and np.abs(g).max() <= 1e-14


@pytest.mark.parametrize("mode", ["stretch", "shear"])
def test_uniform_deformations_closed_form(sheet, mode):
    sc, R = sheet
    b = sc.softs[0]
    h2 = sc.params.dt ** 2
    ks, ksh = b.E, b.E / (2 * (1 + b.nu))
    area = 0.2 ** 2
    y = R.get_state()[0].copy()
    n = R.n_soft_verts
    x = y[:3 * n].reshape(-1, 3).copy()
    for v in (0.7, 1.3):
        xx = x.copy()
        if mode == "stretch":
            xx[:, 0] *= v
            want = h2 * area * 0.5 * ks * (v - 1) ** 2
        else:
            gam = v - 1.0
            xx[:, 0] += gam * x[:, 2]
            want = h2 * area * (0.5 * ks * (np.sqrt(1 + gam ** 2) - 1) ** 2 + 0.5 * ksh * gam ** 2)
        yy = y.copy()
        yy[:3 * n] = xx.ravel()
        assert elastic(R, yy)[0] == pytest.approx(want, rel=1e-12)


def test_gradient_and_hessian(sheet):
    sc, R = sheet
    y0 = R.get_state()[0].copy()
    n = R.n_soft_verts
    rng = np.random.default_rng(3)
    y = y0.copy()
    y[:3 * n] += rng.normal(scale=4e-3, size=3 * n)
    e, g = elastic(R, y)
    h = 1e-7
    gfd = np.zeros(3 * n)
    for i in range(3 * n):
        yp, ym = y.copy(), y.copy()
        yp[i] += h
        ym[i] -= h
        gfd[i] = (elastic(R, yp)[0] - elastic(R, ym)[0]) / (2 * h)
    assert np.abs(gfd - g[:3 * n]).max() <= 1e-6 * np.abs(g).max()
    # projected Hessian: symmetric PSD (columns of H from H e_i)
    R.set_state(y, np.zeros_like(y))
    R.ip_assemble(y, mask=1 << 1)
    H = np.stack([R.hessian_matvec(np.eye(R.n_dof)[i]) for i in range(R.n_dof)], 1)[:3 * n, :3 * n]
    assert np.abs(H - H.T).max() <= 1e-12 * np.abs(H).max()
    assert np.linalg.eigvalsh(H).min() >= -1e-10 * np.abs(H).max()
    # pure stretch along u and v (every part convex): projected = exact Hessian
    x = y0[:3 * n].reshape(-1, 3).copy()
    x[:, 0] *= 1.2
    x[:, 2] *= 1.1
    ys = y0.copy()
    ys[:3 * n] = x.ravel()
    R.set_state(ys, np.zeros_like(ys))
    R.ip_assemble(ys, mask=1 << 1)
    H = np.stack([R.hessian_matvec(np.eye(R.n_dof)[i]) for i in range(R.n_dof)], 1)[:3 * n, :3 * n]
    Hfd = np.zeros((3 * n, 3 * n))
    for i in range(3 * n):
        yp, ym = ys.copy(), ys.copy()
        yp[i] += 1e-6
        ym[i] -= 1e-6
        Hfd[:, i] = (elastic(R, yp)[1][:3 * n] - elastic(R, ym)[1][:3 * n]) / 2e-6
    assert np.abs(Hfd - H).max() <= 1e-6 * np.abs(H).max()


def test_garment_on_cone_stays_intersection_free():
    """The oracle's own steps of the garment dropped onto the fixed cone (free fall, first
    contact with the apex, draping): every step converges, the exact checker finds no
    intersecting (edge, triangle) pair between the sheet and the cone after any step,
    and before contact the sheet falls as a rigid body (each vertex by h^2 g per step
    from rest at the first step, no membrane strain)."""
    from oracle import exact
    sc = sg.garment_on_cone(gap=2e-3, steps=8)
    sc.params.dt = 0.005
    R = ref.RefScene(sc)
    tris, edges, vb = R.surface()
    y0 = R.get_state()[0].copy()
    for k in range(8):
        st = R.step(1)[0]
        assert st["status"] == 0
        y = R.get_state()[0]
        assert exact.count_intersections(R.surface_positions(y), tris, edges, vb) == 0
        if k == 0:
            n = R.n_soft_verts
            d = (y - y0)[:3 * n].reshape(-1, 3)
            g = np.asarray(sc.params.gravity) * sc.params.dt ** 2
            assert np.abs(d - g).max() <= 1e-9 * np.abs(g).max()
