"""Ties between closest-feature types.  The oracle takes the first minimum of its
floating-point feature distances in enumeration order; the library classifies by
Voronoi-region tests, which put a foot point lying exactly on a triangle edge in the
edge's region.  At such a tie the distance and its gradient do not depend on the
choice, but the barrier Hessians do: for the point's own block the edge type adds
kappa b'(d)/d m m^T (m the in-plane normal of the edge; see the oracle pin of typed
pairs), which the PSD projection changes but does not remove.

A soft tet's vertex sits exactly above the diagonal edge shared by the two triangles
of the fixed slab's top face (x = z, exactly representable), at several heights below
dhat.  The oracle's rounding makes the face distance the smaller one for both pairs;
the library takes the edge.  Gates: energy terms and gradients within 1e-9 (unique);
the Hessian is the one of the library's valid choice: the oracle's H v plus, for each
pair at the tie, the oracle's projected (edge - face) block of the point applied to v,
within 1e-9 of |H v|, for v along m (where the choices differ), vertical, and random.
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
    # the pairs at the tie and the point blocks of their (edge - face) Hessians
    dhat = sc.params.dhat
    xs = R.surface_positions(y)
    tris = R.surface()[0]
    pts = R.candidates(xs, None, dhat)[0]
    blocks, oracle_types = [], []
    for v, t in pts:
        x12 = np.concatenate([xs[v], xs[tris[t]].ravel()])
        dist, ty = ref.dist_pt(x12)
        if dist >= dhat:
            continue
        ef, _, Hf = R.pair_energy(0, x12, ftype=6)
        for k in range(3):
            ek, _, Hk = R.pair_energy(0, x12, ftype=3 + k)
            if abs(ek - ef) <= 1e-12 * ef:           # face and edge k at the same distance
                i = [j for j in range(4) if np.array_equal(y[3 * j:3 * j + 3], xs[v])][0]
                assert ty in (6, 3 + k) and i == 0
                oracle_types.append(ty)
                if ty == 6:                           # the oracle's rounding took the face
                    blocks.append((i, (Hk - Hf)[:3, :3]))
    log(f"d = {d}: oracle types at the tie {oracle_types} (6 face, 3-5 edges)")
    assert len(oracle_types) == 2
    m = np.zeros(12)
    m[0], m[2] = 1 / np.sqrt(2), -1 / np.sqrt(2)       # vertex 0 along the in-plane normal of x = z
    rng = np.random.default_rng(int(d * 1e5))
    for v in [m, np.r_[0, 1.0, 0, np.zeros(9)]] + [rng.normal(size=12) for _ in range(3)]:
        hr = R.hessian_matvec(v)
        hx = hr.copy()
        for i, B in blocks:
            hx[3 * i:3 * i + 3] += B @ v[3 * i:3 * i + 3]
        hg = G.hessian_matvec(v).cpu().numpy()
        log(f"d = {d}: |H_gpu v - H_oracle v| {np.abs(hg - hr).max():.3e}, with the edge choice "
            f"{np.abs(hg - hx).max():.3e} (|H v| {np.abs(hx).max():.3e})")
        assert np.abs(hg - hx).max() <= 1e-9 * np.abs(hx).max()
