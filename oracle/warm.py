"""FP64 reference of the learned initial guess's inputs and training target (test
infrastructure only: the test suite, the smoke check and the CPU-baseline leg of the
benchmark use it; the HIP library never does).

The features of soft vertex i at the start of a step, with s = h * 0.05 m/s:
  0-2   h v_i / s;  3-5  h (v_i - v_i^prev) / s;
  6     min(d_i, 4 dhat) / dhat, d_i the distance from x_i to the nearest triangle of
        another body (surface vertices only; 4 otherwise);
  7-9   unit vector from x_i to the closest point of that triangle;
  10-12 h (velocity of that closest point) / s;
  13-15 h (target velocity - velocity) / s of the driven affine body owning it.
Entries 7-15 are zero when no triangle lies within 4 dhat.  Target of a step:
((x^{t+1} - x^t) - h v^t) / s per soft vertex.

The nearest triangle is searched over the candidate pairs of radius 4 dhat (a superset
of every triangle within 4 dhat); among equal distances the first pair in the sorted
candidate list is taken.  The closest point is the textbook region test on the
triangle (Voronoi regions of vertices, edges and face).
"""
from __future__ import annotations

import numpy as np

SPEED = 0.05


def closest_point_triangle(p, a, b, c):
    """Closest point of triangle abc to p and its barycentric weights (wa, wb, wc),
    by the Voronoi-region case analysis of the triangle (vertex, edge, face)."""
    ab, ac, ap = b - a, c - a, p - a
    d1, d2 = ab @ ap, ac @ ap
    if d1 <= 0 and d2 <= 0:
        return a, (1.0, 0.0, 0.0)
    bp = p - b
    d3, d4 = ab @ bp, ac @ bp
    if d3 >= 0 and d4 <= d3:
        return b, (0.0, 1.0, 0.0)
    vc = d1 * d4 - d3 * d2
    if vc <= 0 and d1 >= 0 and d3 <= 0:
        v = d1 / (d1 - d3)
        return a + v * ab, (1.0 - v, v, 0.0)
    cp = p - c
    d5, d6 = ab @ cp, ac @ cp
    if d6 >= 0 and d5 <= d6:
        return c, (0.0, 0.0, 1.0)
    vb = d5 * d2 - d1 * d6
    if vb <= 0 and d2 >= 0 and d6 <= 0:
        w = d2 / (d2 - d6)
        return a + w * ac, (1.0 - w, 0.0, w)
    va = d3 * d6 - d5 * d4
    if va <= 0 and (d4 - d3) >= 0 and (d5 - d6) >= 0:
        w = (d4 - d3) / ((d4 - d3) + (d5 - d6))
        return b + w * (c - b), (0.0, 1.0 - w, w)
    den = 1.0 / (va + vb + vc)
    v, w = vb * den, vc * den
    return a + ab * v + ac * w, (1.0 - v - w, v, w)


def soft_surface_vertices(scene):
    """Soft vertex index of each soft surface vertex, in the surface numbering (the
    boundary vertices of each soft body in ascending order, bodies in order)."""
    out, off = [], 0
    for b in scene.softs:
        faces = np.sort(np.concatenate([b.tets[:, [0, 1, 2]], b.tets[:, [0, 1, 3]], b.tets[:, [0, 2, 3]],
                                        b.tets[:, [1, 2, 3]]]), axis=1)
        uniq, cnt = np.unique(faces, axis=0, return_counts=True)
        out.append(np.unique(uniq[cnt == 1].ravel()) + off)
        off += len(b.rest_pos)
    return np.concatenate(out) if out else np.zeros(0, dtype=np.int64)


def target_velocities(scene, step):
    """Translational target velocity of every affine body over step `step` -> step+1
    (the kinematic target moves at target_vel until target_stop)."""
    h = scene.params.dt
    tnext = (step + 1) * h
    out = np.zeros((len(scene.affines), 3))
    for k, b in enumerate(scene.affines):
        if b.mode != 2:
            continue
        span = min(tnext, b.target_stop) - min(tnext - h, b.target_stop)
        out[k] = np.asarray(b.target_vel, dtype=float) * span / h
    return out


def features(scene, R, y, ydot, ydot_prev, step):
    """Features [n_soft_verts, 16] (FP64) at state (y, ydot) with the previous step's
    velocity ydot_prev; R is the oracle scene of `scene` (surface map and candidates)."""
    p = scene.params
    h, dhat = p.dt, p.dhat
    inv = h / (h * SPEED)
    nsv = R.n_soft_verts
    n3 = 3 * nsv
    F = np.zeros((nsv, 16))
    v = np.asarray(ydot[:n3]).reshape(-1, 3)
    vp = np.asarray(ydot_prev[:n3]).reshape(-1, 3)
    F[:, 0:3] = inv * v
    F[:, 3:6] = inv * (v - vp)
    F[:, 6] = 4.0
    tris, _, vb = R.surface()
    xs = R.surface_positions(y)
    nsoft_bodies = len(scene.softs)
    # surface velocities: the vertex map is linear in y, so mapping ydot gives them for
    # soft and non-fixed affine vertices; fixed bodies do not move
    vs = R.surface_positions(ydot)
    for k, b in enumerate(scene.affines):
        if b.mode == 1:
            vs[vb == nsoft_bodies + k] = 0.0
    # DOF offset of each non-fixed affine body
    dof0, o = {}, n3
    for k, b in enumerate(scene.affines):
        if b.mode != 1:
            dof0[k] = o
            o += 12
    tv = target_velocities(scene, step)
    sv_soft = soft_surface_vertices(scene)
    pt, _ = R.candidates(xs, None, 4.0 * dhat)
    best = {}
    for k, (sv, t) in enumerate(pt):
        if sv >= len(sv_soft):
            continue                                     # an affine vertex
        a, b_, c = tris[t]
        cp, w = closest_point_triangle(xs[sv], xs[a], xs[b_], xs[c])
        d = float(np.linalg.norm(cp - xs[sv]))
        if sv not in best or d < best[sv][0]:
            best[sv] = (d, t, cp, w)
    for sv, (d, t, cp, w) in best.items():
        if not d < 4.0 * dhat:
            continue
        i = sv_soft[sv]
        F[i, 6] = d / dhat
        if d > 0:
            F[i, 7:10] = (cp - xs[sv]) / d
        a, b_, c = tris[t]
        F[i, 10:13] = inv * (w[0] * vs[a] + w[1] * vs[b_] + w[2] * vs[c])
        body = int(vb[a]) - nsoft_bodies
        if body >= 0 and scene.affines[body].mode == 2:
            pd = np.asarray(ydot[dof0[body]:dof0[body] + 3])
            F[i, 13:16] = inv * (tv[body] - pd)
    return F


def warm_target(scene, y_next, y, ydot, nsv):
    """Training target [nsv, 3] of the step y -> y_next taken from velocity ydot."""
    h = scene.params.dt
    n3 = 3 * nsv
    return (((np.asarray(y_next[:n3]) - np.asarray(y[:n3])) - h * np.asarray(ydot[:n3])) / (h * SPEED)).reshape(-1, 3)


def fit_correction(scene, mass, y, corr, mode):
    """Per-soft-body fit of a correction field [nsv, 3] (the learned guess's
    post-processing, a project choice): mode 0 the field itself, 2 its mass-weighted mean
    over each body's vertices, 1 its mass-weighted least-squares affine fit
    cbar + A (x - xbar) at the positions y; a body whose centred second moment S has
    det S <= 1e-9 (tr S)^3 keeps the mean.  `mass`: the lumped vertex masses.  The
    affine fit is solved as a weighted least-squares problem on the design [1, x - xbar]."""
    corr = np.asarray(corr, dtype=np.float64).reshape(-1, 3)
    out = corr.copy()
    if mode == 0:
        return out
    x_all = np.asarray(y, dtype=np.float64)[:3 * len(corr)].reshape(-1, 3)
    v0 = 0
    for body in scene.softs:
        n = len(body.rest_pos)
        w, x, c = mass[v0:v0 + n], x_all[v0:v0 + n], corr[v0:v0 + n]
        W = w.sum()
        xb, cb = w @ x / W, w @ c / W
        out[v0:v0 + n] = cb
        if mode == 1:
            X = x - xb
            S = (X * w[:, None]).T @ X
            if np.linalg.det(S) > 1e-9 * np.trace(S) ** 3:
                D = np.hstack([np.ones((n, 1)), X])
                sw = np.sqrt(w)[:, None]
                coef = np.linalg.lstsq(D * sw, c * sw, rcond=None)[0]
                out[v0:v0 + n] = D @ coef
        v0 += n
    return out

