"""Exact intersection count (test infrastructure only).

Counts inter-body (edge, triangle) pairs whose closed segment and closed triangle
intersect, and tetrahedra with non-positive volume, using exact rational arithmetic
(every FP64 input is exactly a Fraction).  Pairs whose bounding boxes do not overlap
are skipped first with exact float comparisons.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _F(p):
    return tuple(Fraction(float(c)) for c in p)


def _sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def _det3(u, v, w):
    return (u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0])
            + u[2] * (v[0] * w[1] - v[1] * w[0]))


def orient3d(a, b, c, d):
    x = _det3(_sub(b, a), _sub(c, a), _sub(d, a))
    return (x > 0) - (x < 0)


def _orient2d(a, b, c):
    x = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
    return (x > 0) - (x < 0)


def _on_segment2(p, a, b):
    return (min(a[0], b[0]) <= p[0] <= max(a[0], b[0]) and min(a[1], b[1]) <= p[1] <= max(a[1], b[1]))


def _seg_seg2(p, q, a, b):
    o1, o2, o3, o4 = _orient2d(p, q, a), _orient2d(p, q, b), _orient2d(a, b, p), _orient2d(a, b, q)
    if o1 * o2 < 0 and o3 * o4 < 0:
        return True
    if o1 == 0 and _on_segment2(a, p, q):
        return True
    if o2 == 0 and _on_segment2(b, p, q):
        return True
    if o3 == 0 and _on_segment2(p, a, b):
        return True
    if o4 == 0 and _on_segment2(q, a, b):
        return True
    return False


def _in_tri2(p, a, b, c):
    s = [_orient2d(a, b, p), _orient2d(b, c, p), _orient2d(c, a, p)]
    return all(x >= 0 for x in s) or all(x <= 0 for x in s)


def _cross(u, v):
    return (u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0])


def _drop_axis(n):
    """Coordinates kept when projecting onto the plane whose normal is n: the axis
    of n's largest component is dropped, so the projection is one-to-one."""
    ax = max(range(3), key=lambda k: abs(n[k]))
    return [k for k in range(3) if k != ax]


def seg_seg_intersect(p, q, a, b) -> bool:
    """Closed segment pq against closed segment ab in 3-D, exact (Fraction inputs).
    Either segment may be a single point."""
    if orient3d(p, q, a, b) != 0:
        return False                      # not coplanar: skew or apart
    pq, ab, ap = _sub(q, p), _sub(b, a), _sub(p, a)
    for n in (_cross(pq, ab), _cross(pq, _sub(a, p)), _cross(pq, _sub(b, p)), _cross(ab, ap),
              _cross(ab, _sub(q, a))):
        if any(c != 0 for c in n):
            keep = _drop_axis(n)
            p2, q2, a2, b2 = (tuple(v[k] for k in keep) for v in (p, q, a, b))
            return _seg_seg2(p2, q2, a2, b2)
    # all four points on one line (or coincident): overlap of the 1-D intervals along
    # an axis on which the points differ
    diffs = [pq, ab, ap]
    ax = max(range(3), key=lambda k: max(abs(d[k]) for d in diffs))
    lo1, hi1 = min(p[ax], q[ax]), max(p[ax], q[ax])
    lo2, hi2 = min(a[ax], b[ax]), max(a[ax], b[ax])
    return lo1 <= hi2 and lo2 <= hi1


def seg_tri_intersect(p, q, a, b, c) -> bool:
    """Closed segment pq against closed triangle abc, exact.  A degenerate triangle
    (collinear or coincident corners) is the union of its three edges."""
    p, q, a, b, c = map(_F, (p, q, a, b, c))
    n = _cross(_sub(b, a), _sub(c, a))
    if all(x == 0 for x in n):
        return any(seg_seg_intersect(p, q, u, v) for u, v in ((a, b), (b, c), (c, a)))
    s1, s2 = orient3d(a, b, c, p), orient3d(a, b, c, q)
    if s1 * s2 > 0:
        return False
    if s1 == 0 and s2 == 0:
        # coplanar: project along the triangle normal's largest component
        keep = _drop_axis(n)
        p2, q2, a2, b2, c2 = (tuple(v[k] for k in keep) for v in (p, q, a, b, c))
        if _in_tri2(p2, a2, b2, c2) or _in_tri2(q2, a2, b2, c2):
            return True
        return _seg_seg2(p2, q2, a2, b2) or _seg_seg2(p2, q2, b2, c2) or _seg_seg2(p2, q2, c2, a2)
    t = [orient3d(p, q, a, b), orient3d(p, q, b, c), orient3d(p, q, c, a)]
    return all(x >= 0 for x in t) or all(x <= 0 for x in t)


def _boxes(xs, idx):
    P = xs[idx]                         # (n, k, 3)
    return P.min(axis=1), P.max(axis=1)


def count_intersections(xs, tris, edges, vbody) -> int:
    """Inter-body (edge, triangle) pairs that intersect, exactly."""
    xs = np.asarray(xs, dtype=np.float64)
    tris = np.asarray(tris); edges = np.asarray(edges); vbody = np.asarray(vbody)
    tlo, thi = _boxes(xs, tris)
    elo, ehi = _boxes(xs, edges)
    tb = vbody[tris[:, 0]]
    eb = vbody[edges[:, 0]]
    n = 0
    for e in range(len(edges)):
        m = np.all(elo[e] <= thi, axis=1) & np.all(tlo <= ehi[e], axis=1) & (tb != eb[e])
        for t in np.nonzero(m)[0]:
            if seg_tri_intersect(xs[edges[e, 0]], xs[edges[e, 1]], xs[tris[t, 0]], xs[tris[t, 1]], xs[tris[t, 2]]):
                n += 1
    return n


def count_inverted(x, tets) -> int:
    """Tetrahedra with non-positive signed volume, exactly."""
    n = 0
    for t in np.asarray(tets):
        a, b, c, d = (_F(x[i]) for i in t)
        if _det3(_sub(b, a), _sub(c, a), _sub(d, a)) <= 0:
            n += 1
    return n
