"""Seeded synthetic scene generators shared by the oracle tests and the HIP path.

This module only produces raw inputs: rest/initial vertex positions, tetrahedra,
closed triangle surfaces, material constants and solver parameters.  It holds
none of the method's arithmetic (no volumes, masses, surfaces, distances or
energies): each side of the parity tests derives those on its own.

Workloads (stand-ins for the paper's unavailable objects; the paper evaluates on
scanned/dataset objects, here replaced by analytic shapes of the stated sizes):
  * cube_drop()       soft 0.1 m cube, 4^3 cells x 6 tets, dropped from a 5 mm gap
                      onto a fixed affine slab (the material-sensitivity drop of the
                      ablation study, Sec. "Sensitivity of Soft Material Simulation").
  * gripper(seed, r)  soft ellipsoid voxelised on an r^3 grid squeezed by two driven
                      affine finger boxes (the grasp setting of Sec. "Simulation
                      Procedure"/"Parallel Grasp Generation").
  * box_on_cube()     a free affine box falling onto a soft cube resting on a fixed
                      slab (the coupled soft-rigid setting with a free rigid body).
  * batch_scene(i)    uneven grasp scenes: box or ellipsoid at r in 8..32, random
                      material, gripper orientation uniform on SO(3).
"""
from __future__ import annotations

import dataclasses
from collections import deque
from dataclasses import dataclass, field

import numpy as np

MODE_FREE, MODE_FIXED, MODE_DRIVEN = 0, 1, 2
NEO_HOOKEAN, STVK, FIXED_COROTATED, BARAFF_WITKIN = 0, 1, 2, 3
PREC_FP64, PREC_MIXED = 0, 1


@dataclass
class Params:
    dt: float = 0.01
    dhat: float = 1e-3
    kappa: float = 0.0          # <= 0: automatic barrier stiffness
    mu: float = 0.5
    eps_v: float = 1e-3
    gravity: tuple = (0.0, -9.81, 0.0)
    newton_tol: float = 1e-6    # m/s; converged when max vertex |dx| <= newton_tol*dt
    pcg_rtol: float = 1e-4
    ccd_s: float = 0.1
    newton_max: int = 200
    pcg_max: int = 0            # <= 0: number of free DOFs
    precision: int = PREC_FP64
    warm_start: int = 0


@dataclass
class SoftBody:
    rest_pos: np.ndarray        # (n,3) float64
    tets: np.ndarray            # (m,4) int32, positively oriented
    E: float
    nu: float
    rho: float
    pos0: np.ndarray | None = None
    vel0: np.ndarray | None = None
    model: int = NEO_HOOKEAN    # constitutive model: NEO_HOOKEAN, STVK, FIXED_COROTATED or BARAFF_WITKIN
    tris: np.ndarray | None = None  # (k,3) int32 garment triangles (BARAFF_WITKIN: E, nu in N/m, rho kg/m^2)


@dataclass
class AffineBody:
    rest_pos: np.ndarray        # (n,3) float64, world positions at t=0
    tris: np.ndarray            # (k,3) int32, closed, outward
    rho: float = 1000.0
    stiffness: float = 1e8      # orthogonality stiffness (Pa)
    mode: int = MODE_FREE
    qdot0: np.ndarray = field(default_factory=lambda: np.zeros(12))
    kappa_A: float = 0.0
    target_vel: np.ndarray = field(default_factory=lambda: np.zeros(3))
    target_stop: float = 0.0    # seconds after which the driven target is held


@dataclass
class Scene:
    name: str
    params: Params
    softs: list
    affines: list
    n_steps: int
    seed: int | None = None
    meta: dict = field(default_factory=dict)

    def replace_params(self, **kw) -> "Scene":
        return dataclasses.replace(self, params=dataclasses.replace(self.params, **kw))


# ----------------------------------------------------------------------------- meshes

# Freudenthal split of a unit cell: one tet per permutation of the axes, all sharing
# the main diagonal (0,0,0)-(1,1,1).  The tet (0, e_a, e_a+e_b, 1) has the sign of the
# permutation (a,b,c); odd ones get two vertices swapped so every tet is positive.
_PERMS = [((0, 1, 2), 1), ((1, 2, 0), 1), ((2, 0, 1), 1),
          ((0, 2, 1), -1), ((2, 1, 0), -1), ((1, 0, 2), -1)]


def _cell_tets():
    out = []
    for (a, b, c), sgn in _PERMS:
        p0 = (0, 0, 0)
        p1 = [0, 0, 0]; p1[a] = 1
        p2 = list(p1); p2[b] = 1
        p3 = (1, 1, 1)
        t = [p0, tuple(p1), tuple(p2), p3]
        if sgn < 0:
            t[1], t[2] = t[2], t[1]
        out.append(t)
    return out


_CELL_TETS = _cell_tets()


def voxel_mesh(mask: np.ndarray, origin, H: float):
    """Tet mesh of the kept voxels of `mask` (nx,ny,nz) with cell size H.

    Vertices are the grid corners used by kept voxels, numbered in lexicographic
    (i,j,k) order; each voxel is split into 6 positive tets (consistent diagonal)."""
    idx = np.argwhere(mask)
    corners = set()
    for i, j, k in idx:
        for di in (0, 1):
            for dj in (0, 1):
                for dk in (0, 1):
                    corners.add((i + di, j + dj, k + dk))
    corners = sorted(corners)
    vid = {c: n for n, c in enumerate(corners)}
    verts = np.array([[origin[0] + c[0] * H, origin[1] + c[1] * H, origin[2] + c[2] * H]
                      for c in corners], dtype=np.float64)
    tets = []
    for i, j, k in idx:
        for t in _CELL_TETS:
            tets.append([vid[(i + p[0], j + p[1], k + p[2])] for p in t])
    return verts, np.asarray(tets, dtype=np.int32)


def _largest_component(mask: np.ndarray) -> np.ndarray:
    """Largest face-connected component of a voxel mask (ties: first found)."""
    seen = np.zeros_like(mask, dtype=bool)
    best = None
    best_n = 0
    for start in map(tuple, np.argwhere(mask)):
        if seen[start]:
            continue
        comp = []
        dq = deque([start])
        seen[start] = True
        while dq:
            c = dq.popleft()
            comp.append(c)
            for ax in range(3):
                for s in (-1, 1):
                    n = list(c); n[ax] += s; n = tuple(n)
                    if all(0 <= n[d] < mask.shape[d] for d in range(3)) and mask[n] and not seen[n]:
                        seen[n] = True
                        dq.append(n)
        if len(comp) > best_n:
            best, best_n = comp, len(comp)
    out = np.zeros_like(mask, dtype=bool)
    for c in best:
        out[c] = True
    return out


def shape_mesh(shape: str, abc, r: int):
    """Voxelised box or ellipsoid with semi-axes abc, cubic voxel H = 2 max(abc)/r.

    A voxel is kept when its centre is inside the shape; the largest face-connected
    component is kept.  The grid is centred on the origin."""
    a = np.asarray(abc, dtype=np.float64)
    H = 2.0 * float(a.max()) / r
    n = np.maximum(1, np.ceil(2.0 * a / H - 1e-9).astype(int))
    origin = -0.5 * n * H
    ii, jj, kk = np.meshgrid(*(np.arange(n[d]) for d in range(3)), indexing="ij")
    cx = origin[0] + (ii + 0.5) * H
    cy = origin[1] + (jj + 0.5) * H
    cz = origin[2] + (kk + 0.5) * H
    if shape == "ellipsoid":
        mask = (cx / a[0]) ** 2 + (cy / a[1]) ** 2 + (cz / a[2]) ** 2 <= 1.0
    elif shape == "box":
        mask = (np.abs(cx) <= a[0]) & (np.abs(cy) <= a[1]) & (np.abs(cz) <= a[2])
    else:
        raise ValueError(shape)
    mask = _largest_component(mask)
    return voxel_mesh(mask, origin, H)


def box_surface(center, half, n):
    """Closed outward triangle surface of an axis-aligned box, n x n quads per face.

    `n` may be an int or a 3-tuple (quads along x, y, z)."""
    nn = np.array([n, n, n] if np.isscalar(n) else n, dtype=int)
    center = np.asarray(center, dtype=np.float64)
    half = np.asarray(half, dtype=np.float64)
    vid = {}
    verts = []

    def vert(g):
        g = tuple(int(x) for x in g)
        if g not in vid:
            vid[g] = len(verts)
            verts.append([center[d] - half[d] + 2.0 * half[d] * g[d] / nn[d] for d in range(3)])
        return vid[g]

    tris = []
    for ax in range(3):
        u, v = (ax + 1) % 3, (ax + 2) % 3      # (u, v, ax) is a right-handed frame
        for side in (0, 1):
            for i in range(nn[u]):
                for j in range(nn[v]):
                    def g(di, dj):
                        p = [0, 0, 0]
                        p[ax] = side * nn[ax]
                        p[u] = i + di
                        p[v] = j + dj
                        return vert(p)
                    q = [g(0, 0), g(1, 0), g(1, 1), g(0, 1)]
                    if side == 1:   # outward +ax: u x v = +ax
                        tris.append([q[0], q[1], q[2]]); tris.append([q[0], q[2], q[3]])
                    else:           # outward -ax
                        tris.append([q[0], q[2], q[1]]); tris.append([q[0], q[3], q[2]])
    return np.asarray(verts, dtype=np.float64), np.asarray(tris, dtype=np.int32)


def _quat_to_rot(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def uniform_rotation(rng):
    """Shoemake's uniform random unit quaternion -> rotation matrix."""
    u1, u2, u3 = rng.random(3)
    q = (np.sqrt(u1) * np.cos(2 * np.pi * u3), np.sqrt(1 - u1) * np.sin(2 * np.pi * u2),
         np.sqrt(1 - u1) * np.cos(2 * np.pi * u2), np.sqrt(u1) * np.sin(2 * np.pi * u3))
    return _quat_to_rot(q)


# ----------------------------------------------------------------------------- scenes

def cube_drop(n_cells: int = 4, steps: int = 20, model: int = NEO_HOOKEAN) -> Scene:
    """Soft 0.1 m cube (n_cells^3 x 6 tets) 5 mm above a fixed 0.5x0.05x0.5 m slab;
    `model` selects the cube's constitutive model."""
    L = 0.1
    H = L / n_cells
    mask = np.ones((n_cells,) * 3, dtype=bool)
    # the cube is shifted off the slab's top diagonal (x = z) so that no vertex sits
    # exactly on a feature boundary of the slab's triangles
    verts, tets = voxel_mesh(mask, (-L / 2 + 0.0123, 0.005, -L / 2 - 0.0071), H)
    slab_v, slab_t = box_surface((0.0, -0.025, 0.0), (0.25, 0.025, 0.25), 1)
    p = Params(dt=0.01, dhat=1e-3, kappa=0.0, mu=0.5, eps_v=1e-3, newton_tol=1e-6)
    soft = SoftBody(verts, tets, E=1e5, nu=0.4, rho=1000.0, model=model)
    slab = AffineBody(slab_v, slab_t, rho=1000.0, stiffness=1e8, mode=MODE_FIXED)
    return Scene("cube_drop", p, [soft], [slab], steps)


def box_on_cube(n_cells: int = 4, steps: int = 12) -> Scene:
    """Free affine 0.06 m box (0.2 rad about y, off-centre) 4 mm above a soft 0.1 m cube
    that rests 2 mm above a fixed slab: soft-rigid coupling with a free body on both
    sides of the contact."""
    L = 0.1
    H = L / n_cells
    verts, tets = voxel_mesh(np.ones((n_cells,) * 3, dtype=bool), (-L / 2 + 0.0123, 0.002, -L / 2 - 0.0071), H)
    slab_v, slab_t = box_surface((0.0, -0.025, 0.0), (0.25, 0.025, 0.25), 1)
    bv, bt = box_surface((0.0, 0.0, 0.0), (0.03, 0.03, 0.03), 3)
    c, sn = np.cos(0.2), np.sin(0.2)
    rot = np.array([[c, 0.0, sn], [0.0, 1.0, 0.0], [-sn, 0.0, c]])
    bv = bv @ rot.T + np.array([0.0171, 0.002 + L + 0.004 + 0.03, -0.0093])
    p = Params(dt=0.01, dhat=1e-3, kappa=0.0, mu=0.5, eps_v=1e-3, newton_tol=1e-6)
    soft = SoftBody(verts, tets, E=1e5, nu=0.4, rho=1000.0)
    box = AffineBody(bv, bt, rho=500.0, stiffness=1e8, mode=MODE_FREE)
    slab = AffineBody(slab_v, slab_t, rho=1000.0, stiffness=1e8, mode=MODE_FIXED)
    return Scene("box_on_cube", p, [soft], [box, slab], steps)


FINGER_SIZE = (0.01, 0.08, 0.06)     # closing x approach x width (m)
FINGER_QUADS = 10


def _gripper_fingers(obj_verts, dhat, speed, rot=None, offset=0.0, obj_center=None,
                     quads=FINGER_QUADS, travel_frac=0.25):
    """Two driven finger boxes whose inner faces start 2*dhat outside the object's
    extent along the closing axis, closing at `speed` until they have travelled
    2*dhat + travel_frac * extent, then held."""
    R = np.eye(3) if rot is None else rot
    c = np.zeros(3) if obj_center is None else obj_center
    local = (obj_verts - c) @ R                  # object in gripper frame
    x_ext = float(np.max(np.abs(local[:, 0])))
    fx, fy, fz = FINGER_SIZE
    fingers = []
    stop = (2 * dhat + travel_frac * x_ext) / speed
    for side in (-1.0, 1.0):
        # small fixed shift so finger grid lines do not coincide with voxel grid lines
        cen_local = np.array([side * (x_ext + 2 * dhat + fx / 2), offset + 7.1e-4, -3.7e-4])
        v, t = box_surface(cen_local, (fx / 2, fy / 2, fz / 2), (quads, quads, quads))
        v = v @ R.T + c
        vel = R @ np.array([-side * speed, 0.0, 0.0])
        qd = np.zeros(12); qd[:3] = vel
        fingers.append(AffineBody(v, t, rho=1000.0, stiffness=1e8, mode=MODE_DRIVEN,
                                  qdot0=qd, kappa_A=1e8, target_vel=vel, target_stop=stop))
    return fingers, x_ext


def gripper(seed: int = 0, r: int = 32, steps: int = 200, precision: int = PREC_FP64) -> Scene:
    """Soft ellipsoid (semi-axes U[0.03,0.06] m from `seed`) voxelised on an r^3 grid,
    squeezed by two driven affine fingers closing at 0.05 m/s; no ground."""
    rng = np.random.default_rng(seed)
    abc = rng.uniform(0.03, 0.06, 3)
    verts, tets = shape_mesh("ellipsoid", abc, r)
    p = Params(dt=0.005, dhat=1e-3, kappa=0.0, mu=0.8, eps_v=1e-3, newton_tol=1e-6,
               precision=precision)
    fingers, x_ext = _gripper_fingers(verts, p.dhat, 0.05)
    soft = SoftBody(verts, tets, E=5e4, nu=0.45, rho=1000.0)
    return Scene(f"gripper_r{r}_s{seed}", p, [soft], fingers, steps, seed,
                 meta={"abc": abc.tolist(), "r": r, "x_ext": x_ext})


def batch_scene(seed: int, steps: int = 100) -> Scene:
    """One uneven grasp scene: shape, semi-axes, resolution, material, friction,
    gripper rotation and approach offset drawn in that order from `seed`."""
    rng = np.random.default_rng(seed)
    shape = "box" if rng.random() < 0.5 else "ellipsoid"
    abc = rng.uniform(0.03, 0.06, 3)
    r = int(rng.integers(8, 33))
    E = float(np.exp(rng.uniform(np.log(1e4), np.log(1e6))))
    nu = float(rng.uniform(0.3, 0.48))
    mu = float(rng.uniform(0.3, 1.0))
    R = uniform_rotation(rng)
    off = float(rng.uniform(-0.01, 0.01))
    verts, tets = shape_mesh(shape, abc, r)
    p = Params(dt=0.005, dhat=1e-3, kappa=0.0, mu=mu, eps_v=1e-3, newton_tol=1e-6)
    fingers, x_ext = _gripper_fingers(verts, p.dhat, 0.05, rot=R, offset=off)
    soft = SoftBody(verts, tets, E=E, nu=nu, rho=1000.0)
    return Scene(f"batch_s{seed}", p, [soft], fingers, steps, seed,
                 meta={"shape": shape, "abc": abc.tolist(), "r": r, "E": E, "nu": nu,
                       "mu": mu, "offset": off})


def grasp_scene(seed: int = 0, r: int = 10, shape: str = "ellipsoid", rho: float = 400.0, E: float = 5e4,
                nu: float = 0.45, mu: float = 0.8, speed: float = 0.05, quads: int = 4) -> Scene:
    """Grasp evaluation: a soft object (semi-axes U[0.02, 0.03] m from `seed`) resting
    1.5 dhat above a fixed ground slab (top face at y = 0), two driven finger boxes
    0.01 x 0.03 x 0.04 m (closing x vertical x horizontal) on either side along x, inner
    faces 2 dhat outside the object, closing at `speed`; gravity along -y."""
    rng = np.random.default_rng(seed)
    abc = rng.uniform(0.02, 0.03, 3)
    dhat = 1e-3
    verts, tets = shape_mesh(shape, abc, r)
    verts = verts + np.array([0.0, 1.5 * dhat - verts[:, 1].min(), 0.0])
    cy = 0.5 * (verts[:, 1].min() + verts[:, 1].max())
    x_ext = float(np.max(np.abs(verts[:, 0])))
    fx, fy, fz = 0.01, 0.03, 0.04
    fy_c = max(cy, fy / 2 + 2 * dhat) + 3.1e-4          # off the voxel grid lines
    fingers = []
    for side in (-1.0, 1.0):
        v, t = box_surface((side * (x_ext + 2 * dhat + fx / 2), fy_c, -2.3e-4), (fx / 2, fy / 2, fz / 2),
                           (quads, quads, quads))
        vel = np.array([-side * speed, 0.0, 0.0])
        fingers.append(AffineBody(v, t, rho=1000.0, stiffness=1e8, mode=MODE_DRIVEN, kappa_A=1e8,
                                  target_vel=vel, target_stop=1e9))
    ground_v, ground_t = box_surface((0.0, -0.025, 0.0), (0.15, 0.025, 0.15), 1)
    ground = AffineBody(ground_v, ground_t, rho=1000.0, stiffness=1e8, mode=MODE_FIXED)
    p = Params(dt=0.005, dhat=dhat, kappa=0.0, mu=mu, eps_v=1e-3, newton_tol=1e-6)
    soft = SoftBody(verts, tets, E=E, nu=nu, rho=rho)
    return Scene(f"grasp_s{seed}", p, [soft], fingers + [ground], 0, seed,
                 meta={"abc": abc.tolist(), "r": r, "ground_body": 3, "object_body": 0})


def held_box(kappa_A: float = 1e8, mode: int = MODE_DRIVEN, steps: int = 10) -> Scene:
    """A 0.04 m affine box (density 800) under gravity, alone: driven towards its rest
    pose (a kinematic hold with stiffness kappa_A), or free (`mode`); dt = 0.01 s."""
    v, t = box_surface((0.013, 0.2, -0.007), (0.02, 0.02, 0.02), 2)
    p = Params(dt=0.01, dhat=1e-3, kappa=0.0, mu=0.5, eps_v=1e-3, newton_tol=1e-6)
    box = AffineBody(v, t, rho=800.0, stiffness=1e8, mode=mode, kappa_A=kappa_A,
                     target_vel=np.zeros(3), target_stop=0.0)
    return Scene("held_box", p, [], [box], steps)


def slider_scene(speed: float = 0.1, steps: int = 10) -> Scene:
    """A free affine box (0.04 m, density 800) 3 cm above a fixed rail (0.2 x 0.02 x
    0.02 m), moving along the rail's axis x at `speed`, under gravity; the two are not
    in contact (for prismatic-joint tests: joint between body 1 and body 0, axis x)."""
    rv, rt = box_surface((0.0, 0.0, 0.0), (0.1, 0.01, 0.01), (4, 1, 1))
    bv, bt = box_surface((0.0013, 0.05, -0.0007), (0.02, 0.02, 0.02), 2)
    p = Params(dt=0.01, dhat=1e-3, kappa=0.0, mu=0.5, eps_v=1e-3, newton_tol=1e-6)
    qd = np.zeros(12)
    qd[0] = speed
    rail = AffineBody(rv, rt, rho=1000.0, stiffness=1e8, mode=MODE_FIXED)
    box = AffineBody(bv, bt, rho=800.0, stiffness=1e8, mode=MODE_FREE, qdot0=qd)
    return Scene("slider", p, [], [rail, box], steps)


# ----------------------------------------------------------------------------- tiny cases

def two_tets_scene(model: int = NEO_HOOKEAN) -> Scene:
    """A single soft tet resting 2 mm above a fixed unit-ish affine tetra-box; for
    tiny-case tests."""
    v = np.array([[0, 0.002, 0], [0.02, 0.002, 0], [0, 0.022, 0], [0, 0.002, 0.02]], dtype=np.float64)
    t = np.array([[0, 1, 2, 3]], dtype=np.int32)
    slab_v, slab_t = box_surface((0.0, -0.01, 0.0), (0.05, 0.01, 0.05), 1)
    p = Params(dt=0.01, dhat=1e-3, mu=0.5)
    return Scene("two_tets", p, [SoftBody(v, t, E=1e5, nu=0.4, rho=1000.0, model=model)],
                 [AffineBody(slab_v, slab_t, mode=MODE_FIXED)], 10)


def cone_surface(apex, radius: float, height: float, n: int = 16):
    """Closed outward triangle surface of a cone (apex up, base disk at apex - height)
    with n segments around the axis: apex, n base-rim vertices, base centre."""
    apex = np.asarray(apex, dtype=np.float64)
    ang = 2.0 * np.pi * np.arange(n) / n
    rim = np.stack([apex[0] + radius * np.cos(ang), np.full(n, apex[1] - height), apex[2] + radius * np.sin(ang)], 1)
    verts = np.vstack([apex, rim, [apex[0], apex[1] - height, apex[2]]])
    tris = []
    for k in range(n):
        a, b = 1 + k, 1 + (k + 1) % n
        tris.append([0, b, a])          # side, outward
        tris.append([n + 1, a, b])      # base, facing down
    return verts, np.asarray(tris, dtype=np.int32)


def garment_sheet(n: int, side: float, y: float, offset=(0.0, 0.0)):
    """Square sheet of n x n quads (2 triangles each) in the plane y, centred at
    (offset x, offset z); rest material coordinates are its (x, z)."""
    g = np.linspace(-0.5 * side, 0.5 * side, n + 1)
    X, Z = np.meshgrid(g + offset[0], g + offset[1], indexing="ij")
    verts = np.stack([X.ravel(), np.full(X.size, y), Z.ravel()], 1)
    tris = []
    for i in range(n):
        for j in range(n):
            a, b, c, d = i * (n + 1) + j, (i + 1) * (n + 1) + j, (i + 1) * (n + 1) + j + 1, i * (n + 1) + j + 1
            if (i + j) % 2 == 0:
                tris += [[a, b, c], [a, c, d]]
            else:
                tris += [[a, b, d], [b, c, d]]
    return verts, np.asarray(tris, dtype=np.int32)


def garment_on_cone(n: int = 10, side: float = 0.3, gap: float = 5e-3, E: float = 500.0, nu: float = 0.3,
                    rho: float = 0.2, steps: int = 20, offset=(0.013, -0.007)) -> Scene:
    """A Baraff-Witkin garment (n x n quads, side `side` m, stretch stiffness E N/m,
    shear E / (2 (1 + nu)), area density rho kg/m^2) dropped from `gap` above the apex of
    a fixed cone (radius 0.1 m, height 0.15 m); the sheet's centre is offset from the
    axis so that no vertex sits exactly above the apex.  dt = 0.01 s, dhat = 1e-3 m."""
    cv, ct = cone_surface((0.0, 0.0, 0.0), 0.1, 0.15, 24)
    gv, gt = garment_sheet(n, side, gap, offset)
    p = Params(dt=0.01, dhat=1e-3, mu=0.4)
    cloth = SoftBody(gv, np.zeros((0, 4), np.int32), E=E, nu=nu, rho=rho, model=BARAFF_WITKIN, tris=gt)
    return Scene("garment_on_cone", p, [cloth], [AffineBody(cv, ct, mode=MODE_FIXED)], steps)


def random_state_perturbation(n: int, scale: float, seed: int) -> np.ndarray:
    """Seeded Gaussian perturbation (n,3) used to build deformed test states."""
    return np.random.default_rng(seed).normal(0.0, scale, (n, 3))


# ------------------------------------------------------------------ warm-start network inputs

MLP_SHAPES = [(64, 16), (64,), (64, 64), (64,), (64, 64), (64,), (3, 64), (3,)]


def mlp_init(seed: int) -> np.ndarray:
    """Initial parameters of the 16-64-64-64-3 warm-start network as one flat FP32
    vector (W1, b1, W2, b2, W3, b3, W4, b4; W row-major [out][in]): He-uniform weights
    in +-sqrt(6 / fan_in), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            lim = np.sqrt(6.0 / shape[1])
            parts.append(rng.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


def mlp_batch(seed: int, n: int):
    """Seeded synthetic network inputs of the feature ranges: velocity-like entries
    N(0, 1), a clearance in [0, 4], a unit direction, and targets N(0, 0.3)."""
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, 16))
    x[:, 6] = rng.uniform(0.0, 4.0, size=n)
    d = rng.normal(size=(n, 3))
    x[:, 7:10] = d / np.linalg.norm(d, axis=1, keepdims=True)
    t = rng.normal(scale=0.3, size=(n, 3))
    return x.astype(np.float32), t.astype(np.float32)
