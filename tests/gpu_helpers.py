"""Helpers shared by the GPU tests (no method arithmetic)."""
import numpy as np


def scene_topology(B, j, xs):
    """Surface positions, triangles, edges and vertex bodies of scene j of a batch, taken
    from the library's surface view and re-based to the scene's first surface vertex
    (surface vertices are numbered scene by scene)."""
    tris, edges, vb, _ = (t.cpu().numpy() for t in B.surface_view())
    s0, s1 = (int(x) for x in B.layout[j, 6:8])
    t = tris[(tris[:, 0] >= s0) & (tris[:, 0] < s1)] - s0
    e = edges[(edges[:, 0] >= s0) & (edges[:, 0] < s1)] - s0
    return np.ascontiguousarray(xs[s0:s1]), t, e, vb[s0:s1]
