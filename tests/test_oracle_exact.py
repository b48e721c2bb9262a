"""Pins of the exact intersection checker (oracle/exact.py).

The checker decides the intersection-free property the paper claims for every
accepted step (Sec. I and the experiments of Sec. V): an inter-body (edge, triangle)
pair counts when the closed segment and the closed triangle share a point, and a tet
counts when its signed volume is not positive.  The pins below fix that definition
on constructed cases whose answer is known by hand (through the interior, touching
at a vertex, along an edge, one ulp outside an edge, coplanar overlapping and
disjoint, degenerate triangles) and against an independent parametric solve with
rational arithmetic on random integer configurations.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact

TRI = ((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0))
ULP = 2.0 ** -52


def seg(x, y, z0=-1.0, z1=1.0):
    return (x, y, z0), (x, y, z1)


@pytest.mark.parametrize("p,q,expect", [
    (*seg(0.25, 0.25), True),                      # through the interior
    (*seg(2.0, 2.0), False),                       # beside the triangle
    (*seg(0.5, 0.5), True),                        # through the hypotenuse x + y = 1
    (*seg(0.5, 0.5 + ULP), False),                 # one ulp beyond the hypotenuse
    (*seg(0.5, 0.0), True),                        # through the edge y = 0
    (*seg(0.5, -2.0 ** -60), False),               # just below the edge y = 0
    (*seg(0.0, 0.0), True),                        # through a corner
    (*seg(1.0, 0.0), True),                        # through another corner
    (*seg(1.0 + ULP * 2, 0.0), False),             # past that corner
    ((0.2, 0.2, 0.0), (0.2, 0.2, 1.0), True),      # endpoint on the interior
    ((0.2, 0.2, 2 ** -40), (0.2, 0.2, 1.0), False),  # endpoint just above it
    ((0.0, 0.0, 0.0), (-1.0, -1.0, -1.0), True),   # endpoint on a corner
    ((0.5, 0.5, 0.0), (3.0, 3.0, 1.0), True),      # endpoint on the hypotenuse
])
def test_segment_triangle_constructed(p, q, expect):
    assert exact.seg_tri_intersect(p, q, *TRI) is expect
    # symmetric in the segment's ends and in the triangle's orientation
    assert exact.seg_tri_intersect(q, p, *TRI) is expect
    assert exact.seg_tri_intersect(p, q, TRI[0], TRI[2], TRI[1]) is expect


@pytest.mark.parametrize("p,q,expect", [
    ((-1.0, 0.25, 0.0), (2.0, 0.25, 0.0), True),   # coplanar, crossing two edges
    ((0.1, 0.1, 0.0), (0.2, 0.2, 0.0), True),      # coplanar, inside
    ((2.0, 2.0, 0.0), (3.0, 1.5, 0.0), False),     # coplanar, disjoint
    ((-1.0, 0.0, 0.0), (-0.5, 0.0, 0.0), False),   # coplanar, on the line of an edge, apart
    ((-1.0, 0.0, 0.0), (0.0, 0.0, 0.0), True),     # coplanar, touching a corner end to end
    ((-1.0, 1.0, 0.0), (1.0, -1.0, 0.0), True),    # coplanar, touching a corner only
    ((-1.0, 1.0 - ULP, 0.0), (1.0 - ULP, -1.0, 0.0), False),  # ... moved off it: x + y = -ulp
    ((1.0, 1.0, 0.0), (2.0, 0.0, 0.0), False),     # coplanar, parallel to the hypotenuse
    ((0.5, 0.5, 0.0), (2.0, -1.0, 0.0), True),     # coplanar, along the hypotenuse
])
def test_segment_triangle_coplanar(p, q, expect):
    assert exact.seg_tri_intersect(p, q, *TRI) is expect
    assert exact.seg_tri_intersect(q, p, TRI[1], TRI[2], TRI[0]) is expect


@pytest.mark.parametrize("p,q,tri,expect", [
    # collinear corners on the y axis; a skew segment whose projection crosses them
    ((1.0, 0.5, -1.0), (1.0, 0.5, 1.0), ((0, 0, 0), (0, 1, 0), (0, 2, 0)), False),
    ((0.0, 0.5, -1.0), (0.0, 0.5, 1.0), ((0, 0, 0), (0, 1, 0), (0, 2, 0)), True),
    ((-1.0, 2.0, 0.0), (1.0, 2.0, 0.0), ((0, 0, 0), (0, 1, 0), (0, 2, 0)), True),   # through an end
    ((-1.0, 2.5, 0.0), (1.0, 2.5, 0.0), ((0, 0, 0), (0, 1, 0), (0, 2, 0)), False),
    ((0.0, 1.5, 0.0), (0.0, 5.0, 0.0), ((0, 0, 0), (0, 1, 0), (0, 2, 0)), True),    # collinear overlap
    ((0.0, 2.5, 0.0), (0.0, 5.0, 0.0), ((0, 0, 0), (0, 1, 0), (0, 2, 0)), False),   # collinear apart
    # all three corners at one point
    ((-1.0, 0.0, 0.0), (1.0, 0.0, 0.0), ((0, 0, 0), (0, 0, 0), (0, 0, 0)), True),
    ((-1.0, 1e-300, 0.0), (1.0, 1e-300, 0.0), ((0, 0, 0), (0, 0, 0), (0, 0, 0)), False),
])
def test_segment_degenerate_triangle(p, q, tri, expect):
    assert exact.seg_tri_intersect(p, q, *tri) is expect


def _param_solve(p, q, a, b, c):
    """Independent decision for a segment that is not parallel to the triangle's
    plane: solve p + t (q - p) = a + u (b - a) + v (c - a) by Cramer's rule in
    rationals; None when the system is singular."""
    p, q, a, b, c = (tuple(Fraction(float(x)) for x in v) for v in (p, q, a, b, c))
    cols = [tuple(q[i] - p[i] for i in range(3)), tuple(a[i] - b[i] for i in range(3)),
            tuple(a[i] - c[i] for i in range(3))]
    rhs = tuple(a[i] - p[i] for i in range(3))

    def det(m):
        return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[1][0] * (m[0][1] * m[2][2] - m[0][2] * m[2][1])
                + m[2][0] * (m[0][1] * m[1][2] - m[0][2] * m[1][1]))
    D = det(cols)
    if D == 0:
        return None
    t = det([rhs, cols[1], cols[2]]) / D
    u = det([cols[0], rhs, cols[2]]) / D
    v = det([cols[0], cols[1], rhs]) / D
    return 0 <= t <= 1 and u >= 0 and v >= 0 and u + v <= 1


@pytest.mark.parametrize("seed", range(4))
def test_segment_triangle_vs_parametric_solve(seed):
    # small integer coordinates: many touching cases (t, u or v exactly 0 or 1)
    rng = np.random.default_rng(seed)
    n_checked = n_hit = 0
    for _ in range(1500):
        pts = rng.integers(-2, 3, size=(5, 3)).astype(float)
        if seed % 2:
            pts *= 0.375
        expect = _param_solve(*pts)
        if expect is None:
            continue
        assert exact.seg_tri_intersect(*pts) is expect, pts
        n_checked += 1
        n_hit += expect
    assert n_checked > 800 and n_hit > 50


def _tetra_surface(center, scale):
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float) * scale + center
    t = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]], np.int32)
    return v, t


def _two_bodies(c0, c1, s0=1.0, s1=1.0):
    v0, t0 = _tetra_surface(np.asarray(c0, float), s0)
    v1, t1 = _tetra_surface(np.asarray(c1, float), s1)
    xs = np.vstack([v0, v1])
    tris = np.vstack([t0, t1 + 4])
    edges = np.array(sorted({tuple(sorted((t[i], t[(i + 1) % 3]))) for t in tris for i in range(3)}), np.int32)
    vb = np.array([0] * 4 + [1] * 4, np.int32)
    return xs, tris, edges, vb


def test_count_intersections_bodies():
    xs, tris, edges, vb = _two_bodies((0, 0, 0), (5, 0, 0))
    assert exact.count_intersections(xs, tris, edges, vb) == 0
    # same-body pairs never count: one body alone has every edge touching faces
    assert exact.count_intersections(xs[:4], tris[:4], edges[:6], vb[:4]) == 0
    # a small tetrahedron nested inside the large one: no surface crossing
    xs, tris, edges, vb = _two_bodies((0, 0, 0), (0, 0, 0), 1.0, 0.1)
    assert exact.count_intersections(xs, tris, edges, vb) == 0
    # overlapping: some edges of each pierce faces of the other
    xs, tris, edges, vb = _two_bodies((0, 0, 0), (1.0, 0, 0))
    assert exact.count_intersections(xs, tris, edges, vb) > 0
    # touching: the translated copy whose corner 3 lands exactly on corner 0
    xs, tris, edges, vb = _two_bodies((0, 0, 0), (2.0, 2.0, 0.0))
    assert np.array_equal(xs[7], xs[0])
    assert exact.count_intersections(xs, tris, edges, vb) > 0


def test_count_inverted():
    x = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    assert exact.count_inverted(x, [[0, 1, 2, 3]]) == 0
    assert exact.count_inverted(x, [[0, 2, 1, 3]]) == 1
    flat = x.copy(); flat[3] = [0.5, 0.5, 0.0]
    assert exact.count_inverted(flat, [[0, 1, 2, 3]]) == 1       # zero volume counts
    tiny = x.copy(); tiny[3] = [0.0, 0.0, 2.0 ** -1000]
    assert exact.count_inverted(tiny, [[0, 1, 2, 3]]) == 0       # positive, however small
