"""Pins of the oracle's distance, barrier and PSD-projection routines.

Distances: closed-primitive distance checked against dense sampling of the two
primitives (an upper bound that converges to the true minimum) and against closed
forms.  Barrier: the log barrier of Sec. III (fifth equation) and its C^2 end at
d-hat.  Projection: the nearest PSD matrix in Frobenius norm equals numpy's
eigh-based clamp.
"""
import numpy as np
import pytest

from oracle import ref


def _sample_tri(n):
    u, v = np.meshgrid(np.linspace(0, 1, n), np.linspace(0, 1, n), indexing="ij")
    m = u + v <= 1.0
    return np.stack([1 - u[m] - v[m], u[m], v[m]], axis=1)


def brute_pt(x12, n=400):
    p = x12[:3]
    t = x12[3:].reshape(3, 3)
    pts = _sample_tri(n) @ t
    return np.sqrt(((pts - p) ** 2).sum(1)).min()


def brute_ee(x12, n=1500):
    a0, a1, b0, b1 = x12.reshape(4, 3)
    s = np.linspace(0, 1, n)
    A = a0 + s[:, None] * (a1 - a0)
    B = b0 + s[:, None] * (b1 - b0)
    d2 = ((A[:, None, :] - B[None, :, :]) ** 2).sum(-1)
    return np.sqrt(d2.min())


@pytest.mark.parametrize("seed", range(40))
def test_pt_distance_vs_sampling(seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=12)
    d, t = ref.dist_pt(x)
    b = brute_pt(x)
    # the sampled minimum is an upper bound within the grid spacing
    diam = np.ptp(x[3:].reshape(3, 3), axis=0).max()
    assert d <= b + 1e-12
    assert b - d <= 2 * diam / 400 + 1e-12
    assert 0 <= t <= 6


@pytest.mark.parametrize("seed", range(40))
def test_ee_distance_vs_sampling(seed):
    rng = np.random.default_rng(100 + seed)
    x = rng.normal(size=12)
    d, t = ref.dist_ee(x)
    b = brute_ee(x)
    L = max(np.linalg.norm(x[3:6] - x[:3]), np.linalg.norm(x[9:] - x[6:9]))
    assert d <= b + 1e-12
    assert b - d <= 2 * L / 1500 + 1e-12
    assert 0 <= t <= 8


def test_point_above_triangle_interior():
    t0, t1, t2 = np.array([0., 0, 0]), np.array([1., 0, 0]), np.array([0., 1, 0])
    p = np.array([0.2, 0.3, 0.7])
    d, ty = ref.dist_pt(np.concatenate([p, t0, t1, t2]))
    n = np.cross(t1 - t0, t2 - t0); n /= np.linalg.norm(n)
    assert ty == 6
    assert abs(d - abs(n @ (p - t0))) < 1e-15


def test_pt_types_regions():
    T = [0., 0, 0, 1, 0, 0, 0, 1, 0]
    assert ref.dist_pt(np.array([-1., -1, 0.5] + T))[1] == 0          # nearest vertex t0
    assert ref.dist_pt(np.array([0.5, -1., 0.5] + T))[1] == 3          # edge t0t1
    assert abs(ref.dist_pt(np.array([0.5, -1., 0.] + T))[0] - 1.0) < 1e-15


def test_ee_parallel_and_crossing():
    # parallel edges: distance is the line separation
    x = np.array([0, 0, 0, 1, 0, 0, 0.2, 0.5, 0, 0.8, 0.5, 0], dtype=float)
    assert abs(ref.dist_ee(x)[0] - 0.5) < 1e-15
    # skew edges crossing above each other at height h
    h = 1e-4
    x = np.array([-1, 0, 0, 1, 0, 0, 0, -1, h, 0, 1, h], dtype=float)
    d, t = ref.dist_ee(x)
    assert t == 8 and abs(d - h) < 1e-18


def test_barrier_closed_forms():
    dh = 1e-3
    b = ref.barrier(dh, dh)
    assert np.all(b == 0.0)
    # C^2 at dhat: one-sided limits tend to zero
    b = ref.barrier(dh * (1 - 1e-7), dh)
    assert abs(b[0]) < 1e-20 and abs(b[1]) < 1e-16 and abs(b[2]) < 1e-6
    b = ref.barrier(dh / 2, dh)
    assert abs(b[1] - (-dh * (np.log(2) + 0.5))) < 1e-18
    assert abs(b[0] - (-(dh / 2) ** 2 * np.log(0.5))) < 1e-20
    assert ref.barrier(1e-12, dh)[0] > ref.barrier(1e-9, dh)[0] > 0  # grows to +inf at 0


@pytest.mark.parametrize("d", [1e-6, 1e-4, 5e-4, 9e-4])
def test_barrier_derivatives_fd(d):
    dh = 1e-3
    eps = 1e-4 * min(d, dh - d)
    b = ref.barrier(d, dh)
    bp = ref.barrier(d + eps, dh)
    bm = ref.barrier(d - eps, dh)
    assert abs((bp[0] - bm[0]) / (2 * eps) - b[1]) <= 1e-6 * abs(b[1])
    assert abs((bp[1] - bm[1]) / (2 * eps) - b[2]) <= 1e-6 * abs(b[2])


@pytest.mark.parametrize("n,seed", [(3, 0), (9, 1), (12, 2), (12, 3)])
def test_projection_matches_eigh_clamp(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n)); A = A + A.T
    P = ref.project_psd(A)
    w, V = np.linalg.eigh(A)
    Q = (V * np.maximum(w, 0)) @ V.T
    assert np.abs(P - Q).max() <= 1e-12 * np.abs(A).max()
    # PSD input is left unchanged
    B = A @ A.T
    assert np.abs(ref.project_psd(B) - B).max() <= 1e-12 * np.abs(B).max()
