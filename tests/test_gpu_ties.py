"""Ties between closest-feature types (the oracle takes the first minimum in its
enumeration order; the library classifies by Voronoi regions, so at an exact tie the
two may pick different features).

A soft tet's vertex sits exactly above the diagonal edge shared by the two triangles
of the fixed slab's top face (x = z, exactly representable), at several heights below
dhat: for both point-triangle pairs the point's projection lies on the triangle's
boundary, so "face" and "edge" are both closest features.  The distance and its
gradient are the same for either choice; the unprojected barrier Hessians differ by
kappa b'(d)/d m m^T (m the in-plane normal of the edge), which is negative since
b' < 0 and is removed by the PSD projection, so the projected Hessians coincide.  The
gates: energy terms and gradients within 1e-9, H v within 1e-9 of |H v| for random v
and for v along m (the direction where the unprojected choices differ).
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


@pytest.mark.parametrize("d", [2e-4, 5e-4, 9e-4])
def test_point_above_shared_triangle_edge(zema, d):
    sc = sg.two_tets_scene()
    R = ref.RefScene(sc)
    G = zema.Scene(sc)
    y = np.array([0.01, d, 0.01, 0.03, d + 0.0025, 0.01, 0.01, d + 0.0225, 0.01, 0.01, d + 0.0025, 0.03])
    yd = np.zeros_like(y)
    kappa = R.get_state()[2]
    for S in (R, G):
        S.set_state(y, yd, kappa, 0)
    tr, gr = R.ip_assemble(y)
    tg, gg = G.ip_assemble(y)
    assert tr[4] > 0 and tr[7] == pytest.approx(d, rel=1e-12)
    for k in range(7):
        assert abs(tg[k] - tr[k]) <= 1e-9 * abs(tr[k]) + 1e-15 * abs(tr[6]), k
    assert np.abs(gg.cpu().numpy() - gr).max() <= 1e-9 * np.abs(gr).max()
    m = np.zeros(12)
    m[0], m[2] = 1 / np.sqrt(2), -1 / np.sqrt(2)       # vertex 0 along the in-plane normal of x = z
    rng = np.random.default_rng(int(d * 1e5))
    for v in [m, np.r_[0, 1.0, 0, np.zeros(9)]] + [rng.normal(size=12) for _ in range(3)]:
        hr = R.hessian_matvec(v)
        hg = G.hessian_matvec(v).cpu().numpy()
        assert np.abs(hg - hr).max() <= 1e-9 * np.abs(hr).max()
    log(f"d = {d}: barrier {tr[4]:.3e}, H m (vertex 0) {R.hessian_matvec(m)[:3]}")
