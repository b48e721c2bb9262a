"""Pins of the oracle's constitutive models (Sec. IV-D: neo-Hookean with the
logarithmic volume term, Saint Venant-Kirchhoff, fixed corotated), each checked
against what its definition fixes independently of the implementation:
  * zero energy and gradient at rest and under a rigid rotation;
  * closed forms on F = R diag(s) Q^T: StVK mu sum((s^2-1)/2)^2 + lambda/2 (sum (s^2-1)/2)^2,
    fixed corotated mu sum(s-1)^2 + lambda/2 (s1 s2 s3 - 1)^2, neo-Hookean
    mu/2 (sum s^2 - 3) - mu log J + lambda/2 (log J)^2 (rotations must drop out);
  * the small-strain limit Psi(I + eps H) / eps^2 -> mu |sym H|^2 + lambda/2 (tr H)^2
    (linear elasticity with the same Lame parameters) for every model;
  * gradient and unprojected Hessian against central differences of the energy;
  * the projected Hessian is symmetric PSD and equals the unprojected one where that
    is PSD.
The element is the single tet of the two-tet scene (rest edges 0.02 m along the
axes, so F is the deformation of the edge vectors); its energy is h^2 V Psi(F).
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import ref

MODELS = {"neo-Hookean": sg.NEO_HOOKEAN, "StVK": sg.STVK, "fixed corotated": sg.FIXED_COROTATED}


def rot(axis, ang):
    a = np.asarray(axis, float)
    a /= np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


class Elem:
    def __init__(self, model):
        self.sc = sg.two_tets_scene(model)
        self.R = ref.RefScene(self.sc)
        b = self.sc.softs[0]
        self.X = b.rest_pos
        self.mu = b.E / (2 * (1 + b.nu))
        self.lam = b.E * b.nu / ((1 + b.nu) * (1 - 2 * b.nu))
        Lh = 0.02
        self.c = self.sc.params.dt ** 2 * Lh ** 3 / 6.0      # h^2 V

    def x12(self, F):
        X0 = self.X[0]
        return np.concatenate([X0 + F @ (xa - X0) for xa in self.X])

    def energy(self, F, project=True):
        return self.R.tet_energy(0, self.x12(F), project)

    def psi(self, F):
        return self.energy(F)[0] / self.c


@pytest.fixture(scope="module", params=list(MODELS))
def elem(request):
    return request.param, Elem(MODELS[request.param])


def closed_form(name, mu, lam, s):
    if name == "StVK":
        e = (s ** 2 - 1) / 2
        return mu * np.sum(e ** 2) + 0.5 * lam * np.sum(e) ** 2
    if name == "fixed corotated":
        return mu * np.sum((s - 1) ** 2) + 0.5 * lam * (np.prod(s) - 1) ** 2
    J = np.prod(s)
    return 0.5 * mu * (np.sum(s ** 2) - 3) - mu * np.log(J) + 0.5 * lam * np.log(J) ** 2


def test_rest_and_rigid_rotation_are_free(elem):
    name, E = elem
    scale = E.c * E.mu
    for F in (np.eye(3), rot([1, 2, 3], 0.7), rot([-1, 0.3, 0.2], 2.9)):
        e, g, _ = E.energy(F)
        assert abs(e) <= 1e-12 * scale, (name, e)
        assert np.abs(g).max() <= 1e-10 * scale / 0.02, (name, np.abs(g).max())


@pytest.mark.parametrize("s", [(1.2, 0.9, 1.05), (0.7, 0.8, 1.3), (1.5, 1.0, 1.0)])
def test_closed_form_in_singular_values(elem, s):
    name, E = elem
    s = np.array(s)
    for R, Q in ((np.eye(3), np.eye(3)), (rot([1, 1, 0], 0.4), rot([0, 1, 2], -1.1))):
        F = R @ np.diag(s) @ Q.T
        want = closed_form(name, E.mu, E.lam, s)
        assert E.psi(F) == pytest.approx(want, rel=1e-10), (name, s)


def test_small_strain_limit_is_linear_elasticity(elem):
    name, E = elem
    H = np.array([[0.3, -0.2, 0.1], [0.4, -0.1, 0.25], [-0.15, 0.05, 0.2]])
    S = 0.5 * (H + H.T)
    lin = E.mu * np.sum(S * S) + 0.5 * E.lam * np.trace(H) ** 2
    errs = []
    for eps in (1e-2, 1e-3, 1e-4):
        errs.append(abs(E.psi(np.eye(3) + eps * H) / eps ** 2 - lin) / lin)
    assert errs[-1] < 1e-3, (name, errs)
    assert errs[2] < errs[0]


def test_gradient_and_hessian_against_differences(elem):
    name, E = elem
    rng = np.random.default_rng(5)
    F = np.eye(3) + 0.15 * rng.normal(size=(3, 3))
    assert np.linalg.det(F) > 0
    x = E.x12(F)
    e0, g, H = E.R.tet_energy(0, x, False)
    hstep = 1e-7
    gf = np.zeros(12)
    Hf = np.zeros((12, 12))
    for k in range(12):
        d = np.zeros(12)
        d[k] = hstep
        ep, gp, _ = E.R.tet_energy(0, x + d, False)
        em, gm, _ = E.R.tet_energy(0, x - d, False)
        gf[k] = (ep - em) / (2 * hstep)
        Hf[:, k] = (gp - gm) / (2 * hstep)
    assert np.abs(g - gf).max() <= 1e-6 * np.abs(g).max(), name
    assert np.abs(H - Hf).max() <= 1e-6 * np.abs(H).max(), name


def test_projected_hessian_is_psd(elem):
    """The projection clamps the negative eigenvalues of d2Psi/dF2, so the projected
    element Hessian is symmetric PSD and exceeds the unprojected one by a PSD matrix
    (h^2 V B^T (P - d2Psi/dF2) B with P - d2Psi/dF2 = the clamped negative part)."""
    name, E = elem
    rng = np.random.default_rng(9)
    n = 0
    for trial in range(6):
        F = np.diag([0.55, 1.3, 0.9]) @ rot(rng.normal(size=3), 1.0) + 0.1 * rng.normal(size=(3, 3))
        if np.linalg.det(F) <= 0:
            continue
        n += 1
        _, _, Hp = E.energy(F, project=True)
        _, _, Hu = E.energy(F, project=False)
        top = np.abs(Hp).max()
        assert np.abs(Hp - Hp.T).max() <= 1e-12 * top
        w = np.linalg.eigvalsh(Hp)
        assert w.min() >= -1e-10 * w.max(), (name, w.min(), w.max())
        wd = np.linalg.eigvalsh(0.5 * ((Hp - Hu) + (Hp - Hu).T))
        assert wd.min() >= -1e-10 * top, (name, wd.min())
    assert n >= 3


def test_inverted_element_is_infeasible(elem):
    name, E = elem
    e, _, _ = E.energy(np.diag([1.0, 1.0, -0.5]))
    assert e == float("inf"), name
