"""Pins of the oracle's scene preprocessing and candidate sets.

Affine mass properties against the box closed form (M_b = int rho J^T J, Sec. III
eq. 2), lumped mass against rho * total volume, the cube's boundary surface against
Euler's formula, and the candidate set against brute-force distances over every
inter-body pair (superset of the contact set C of Sec. III eq. 4).
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import ref


def test_box_mass_properties():
    a, b, c = 0.1, 0.04, 0.06
    v, t = sg.box_surface((0.01, -0.02, 0.03), (a / 2, b / 2, c / 2), 3)
    s = sg.Scene("box", sg.Params(), [], [sg.AffineBody(v, t, rho=700.0, mode=sg.MODE_FREE)], 1)
    R = ref.RefScene(s)
    pr = R.affine_props()[0]
    V, m, cen, S = pr[0], pr[1], pr[2:5], pr[5:].reshape(3, 3)
    assert abs(V - a * b * c) < 1e-15
    assert abs(m - 700 * a * b * c) < 1e-12
    assert np.allclose(cen, [0.01, -0.02, 0.03], atol=1e-15)
    S_ref = m * np.diag([a * a, b * b, c * c]) / 12
    assert np.abs(S - S_ref).max() <= 1e-12 * np.abs(S_ref).max()


def test_cube_surface_and_mass():
    s = sg.cube_drop()
    R = ref.RefScene(s)
    tris, edges, vb = R.surface()
    soft = vb == 0
    n_v = soft.sum()
    soft_t = soft[tris[:, 0]]
    soft_e = soft[edges[:, 0]]
    assert (n_v, soft_t.sum(), soft_e.sum()) == (98, 192, 288)
    assert n_v - soft_e.sum() + soft_t.sum() == 2            # Euler characteristic
    assert abs(R.lumped_mass().sum() - 1000.0 * 0.1 ** 3) < 1e-14
    # canonical numbering: smallest id first, sorted triangles, sorted edges a<b
    assert np.all(tris[:, 0] < tris[:, 1]) and np.all(tris[:, 0] < tris[:, 2])
    assert np.all(np.diff(tris[:, 0]) >= 0)
    assert np.all(edges[:, 0] < edges[:, 1])
    # outward orientation: the soft surface encloses +volume
    xs = R.surface_positions(R.get_state()[0])
    T = xs[tris[soft_t]]
    vol = np.einsum("ij,ij->i", T[:, 0], np.cross(T[:, 1], T[:, 2])).sum() / 6
    assert abs(vol - 1e-3) < 1e-15


def _inter_body_distances(R, xs):
    tris, edges, vb = R.surface()
    pt, ee = [], []
    for v in range(R.n_surf):
        for t in range(R.n_tris):
            if vb[v] == vb[tris[t, 0]]:
                continue
            d, _ = ref.dist_pt(np.concatenate([xs[v], xs[tris[t]].ravel()]))
            pt.append((v, t, d))
    for a in range(R.n_edges):
        for b in range(a + 1, R.n_edges):
            if vb[edges[a, 0]] == vb[edges[b, 0]]:
                continue
            d, _ = ref.dist_ee(np.concatenate([xs[edges[a]].ravel(), xs[edges[b]].ravel()]))
            ee.append((a, b, d))
    return pt, ee


def test_candidates_superset_of_contact_set():
    s = sg.cube_drop()
    R = ref.RefScene(s)
    R.step(3)
    y = R.get_state()[0]
    xs = R.surface_positions(y)
    pt, ee = R.candidates(xs)
    tris, edges, vb = R.surface()
    bpt, bee = _inter_body_distances(R, xs)
    need_pt = {(v, t) for v, t, d in bpt if d < s.params.dhat}
    need_ee = {(a, b) for a, b, d in bee if d < s.params.dhat}
    assert len(need_pt) > 0 and len(need_ee) > 0
    assert need_pt <= set(map(tuple, pt))
    assert need_ee <= set(map(tuple, ee))
    # sorted, inter-body, a < b
    assert np.all(np.diff(pt[:, 0] * 10 ** 6 + pt[:, 1]) > 0)
    assert np.all(np.diff(ee[:, 0] * 10 ** 6 + ee[:, 1]) > 0)
    assert np.all(ee[:, 0] < ee[:, 1])
    assert np.all(vb[pt[:, 0]] != vb[tris[pt[:, 1], 0]])
    assert np.all(vb[edges[ee[:, 0], 0]] != vb[edges[ee[:, 1], 0]])


def test_candidate_predicate_is_the_aabb_overlap():
    """Each reported pair's inflated swept boxes overlap and at least one absent
    inter-body pair is separated (the set is exactly the box predicate)."""
    s = sg.cube_drop()
    R = ref.RefScene(s)
    y = R.get_state()[0]
    xs0 = R.surface_positions(y)
    xs1 = xs0 + np.array([0.0, -0.0049, 0.0]) * (np.arange(R.n_surf)[:, None] < 98)
    r = 2e-4
    pt, ee = R.candidates(xs0, xs1, r)
    tris, edges, vb = R.surface()
    lo = np.minimum(xs0, xs1) - r
    hi = np.maximum(xs0, xs1) + r

    def box(idx):
        return lo[idx].min(0), hi[idx].max(0)

    got = set(map(tuple, pt))
    for v in range(R.n_surf):
        for t in range(R.n_tris):
            if vb[v] == vb[tris[t, 0]]:
                continue
            l1, h1 = box([v]); l2, h2 = box(tris[t])
            ov = bool(np.all(l1 <= h2) and np.all(l2 <= h1))
            assert ov == ((v, t) in got)
    assert len(got) > 0
