"""ctypes binding of the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark use
this module.  It loads `libzema_ref.so` (built from `zema_ref.cpp` by `build.py`),
which shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

D = C.c_double
I32 = C.c_int32
I64 = C.c_int64
PD = C.POINTER(C.c_double)
PI32 = C.POINTER(C.c_int32)
PI64 = C.POINTER(C.c_int64)


class Params(C.Structure):
    _fields_ = [("dt", D), ("dhat", D), ("kappa", D), ("mu", D), ("eps_v", D),
                ("gravity", D * 3), ("newton_tol", D), ("pcg_rtol", D), ("ccd_s", D),
                ("newton_max", I32), ("pcg_max", I32), ("precision", I32), ("warm_start", I32)]


class SoftDesc(C.Structure):
    _fields_ = [("n_verts", I32), ("n_tets", I32), ("rest_pos", PD), ("tets", PI32),
                ("pos0", PD), ("vel0", PD), ("E", D), ("nu", D), ("rho", D), ("model", I32), ("pad_", I32),
                ("tris", PI32), ("n_tris", I32), ("pad2_", I32)]


class AffineDesc(C.Structure):
    _fields_ = [("n_verts", I32), ("n_tris", I32), ("rest_pos", PD), ("tris", PI32),
                ("rho", D), ("stiffness", D), ("qdot0", D * 12), ("mode", I32), ("pad_", I32),
                ("kappa_A", D), ("target_vel", D * 3), ("target_stop", D)]


class StepStats(C.Structure):
    _fields_ = [("status", I32), ("newton_iters", I32), ("pcg_iters", I32), ("ls_backtracks", I32),
                ("n_pt_active", I32), ("n_ee_active", I32), ("n_pt_cand", I32), ("n_ee_cand", I32),
                ("al_updates", I32), ("pad_", I32),
                ("alpha_ccd_min", D), ("kappa", D), ("d_min", D), ("energy", D)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "libzema_ref.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        L.zref_scene_create.argtypes = [C.POINTER(Params), C.POINTER(SoftDesc), I32,
                                        C.POINTER(AffineDesc), I32, C.POINTER(C.c_void_p)]
        L.zref_scene_destroy.argtypes = [C.c_void_p]
        L.zref_last_error.argtypes = [C.c_void_p]
        L.zref_last_error.restype = C.c_char_p
        L.zref_set_threads.argtypes = [I32]
        for name, args in [
            ("zref_sizes", [C.c_void_p, PI64]),
            ("zref_surface", [C.c_void_p, PI32, PI32, PI32]),
            ("zref_lumped_mass", [C.c_void_p, PD]),
            ("zref_affine_props", [C.c_void_p, PD]),
            ("zref_set_state", [C.c_void_p, PD, PD, D, I32]),
            ("zref_get_state", [C.c_void_p, PD, PD, PD, PI32]),
            ("zref_set_kappa", [C.c_void_p, D]),
            ("zref_surface_positions", [C.c_void_p, PD, PD]),
            ("zref_candidates", [C.c_void_p, PD, PD, D, PI32, I64, PI64, PI32, I64, PI64]),
            ("zref_ip_assemble", [C.c_void_p, PD, C.c_uint32, PD, PD]),
            ("zref_hessian_matvec", [C.c_void_p, PD, PD]),
            ("zref_pcg_solve", [C.c_void_p, PD, PD, D, I32, PI32, PD]),
            ("zref_ccd_max_step", [C.c_void_p, PD, PD, PD]),
            ("zref_friction_count", [C.c_void_p, PI64]),
            ("zref_friction_table", [C.c_void_p, PI32, PD]),
            ("zref_step", [C.c_void_p, I32, C.POINTER(StepStats)]),
            ("zref_contact_forces", [C.c_void_p, PD, PD]),
            ("zref_set_drive_target", [C.c_void_p, I32, PD]),
            ("zref_set_springs", [C.c_void_p, I32, PI32, PD, PD]),
            ("zref_kinematic_al", [C.c_void_p, D, I32, PD]),
            ("zref_set_prismatic_joints", [C.c_void_p, I32, PI32, PD, PD]),
            ("zref_record", [C.c_void_p, I32]),
            ("zref_record_count", [C.c_void_p, PI64]),
            ("zref_record_get", [C.c_void_p, I64, PI32, PD, PD, PD, PD, PD]),
            ("zref_barrier", [D, D, PD]),
            ("zref_pair_energy", [C.c_void_p, I32, PD, PD, PD, PD, PD, I32]),
            ("zref_pair_energy_typed", [C.c_void_p, I32, PD, PD, I32, PD, PD, PD, I32]),
            ("zref_tet_energy", [C.c_void_p, I32, PD, PD, PD, PD, I32]),
            ("zref_project_psd", [I32, PD, PD]),
            ("zref_accd_pair", [I32, PD, PD, D, PD]),
        ]:
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.zref_dist_pt.argtypes = [PD, PI32]
        L.zref_dist_pt.restype = D
        L.zref_dist_ee.argtypes = [PD, PI32]
        L.zref_dist_ee.restype = D
        _LIB = L
    return _LIB


def _pd(a):
    return a.ctypes.data_as(PD) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> int:
    return lib().zref_set_threads(int(n))


def dist_pt(x12):
    t = I32()
    d = lib().zref_dist_pt(_pd(_f64(x12)), C.byref(t))
    return d, t.value


def dist_ee(x12):
    t = I32()
    d = lib().zref_dist_ee(_pd(_f64(x12)), C.byref(t))
    return d, t.value


def barrier(d, dhat):
    out = np.zeros(3)
    lib().zref_barrier(d, dhat, _pd(out))
    return out


def accd_pair(kind, x12, p12, s=0.1):
    t = D()
    rc = lib().zref_accd_pair(int(kind), _pd(_f64(x12)), _pd(_f64(p12)), float(s), C.byref(t))
    if rc != 0:
        raise OracleError(rc, "intersecting pair at CCD start")
    return t.value


def project_psd(A):
    A = _f64(A)
    out = np.zeros_like(A)
    lib().zref_project_psd(A.shape[0], _pd(A), _pd(out))
    return out


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle status {code}: {msg}")
        self.code = code


class RefScene:
    """Oracle scene built from a `scenegen.Scene`."""

    def __init__(self, scene):
        L = lib()
        self._keep = []
        p = scene.params
        P = Params(p.dt, p.dhat, p.kappa, p.mu, p.eps_v, (D * 3)(*p.gravity), p.newton_tol,
                   p.pcg_rtol, p.ccd_s, p.newton_max, p.pcg_max, p.precision, p.warm_start)
        softs = (SoftDesc * max(1, len(scene.softs)))()
        for k, b in enumerate(scene.softs):
            rp = _f64(b.rest_pos); tt = np.ascontiguousarray(b.tets, dtype=np.int32)
            p0 = _f64(b.pos0) if b.pos0 is not None else None
            v0 = _f64(b.vel0) if b.vel0 is not None else None
            tr = getattr(b, "tris", None)
            tr = np.ascontiguousarray(tr, dtype=np.int32).reshape(-1, 3) if tr is not None else None
            self._keep += [rp, tt, p0, v0, tr]
            softs[k] = SoftDesc(len(rp), len(tt), _pd(rp), tt.ctypes.data_as(PI32), _pd(p0), _pd(v0),
                                b.E, b.nu, b.rho, getattr(b, "model", 0), 0,
                                tr.ctypes.data_as(PI32) if tr is not None else None,
                                len(tr) if tr is not None else 0, 0)
        affs = (AffineDesc * max(1, len(scene.affines)))()
        for k, b in enumerate(scene.affines):
            rp = _f64(b.rest_pos); tt = np.ascontiguousarray(b.tris, dtype=np.int32)
            self._keep += [rp, tt]
            affs[k] = AffineDesc(len(rp), len(tt), _pd(rp), tt.ctypes.data_as(PI32), b.rho, b.stiffness,
                                 (D * 12)(*np.asarray(b.qdot0, dtype=float)), b.mode, 0, b.kappa_A,
                                 (D * 3)(*np.asarray(b.target_vel, dtype=float)), b.target_stop)
        h = C.c_void_p()
        rc = L.zref_scene_create(C.byref(P), softs, len(scene.softs), affs, len(scene.affines), C.byref(h))
        if rc != 0:
            raise OracleError(rc, "scene create failed")
        self.h = h
        self.n_soft_bodies = len(scene.softs)
        s = np.zeros(8, dtype=np.int64)
        L.zref_sizes(self.h, s.ctypes.data_as(PI64))
        (self.n_dof, self.n_soft_verts, self.n_tets, self.n_surf, self.n_tris, self.n_edges,
         self.n_free_bodies, self.n_bodies) = [int(x) for x in s]
        self.params = p

    def __del__(self):
        if getattr(self, "h", None):
            try:
                lib().zref_scene_destroy(self.h)
            except Exception:  # interpreter shutdown: module globals already gone
                pass
            self.h = None

    def _chk(self, rc):
        if rc != 0:
            raise OracleError(rc, lib().zref_last_error(self.h).decode())

    # topology
    def surface(self):
        tris = np.zeros((self.n_tris, 3), dtype=np.int32)
        edges = np.zeros((self.n_edges, 2), dtype=np.int32)
        vb = np.zeros(self.n_surf, dtype=np.int32)
        lib().zref_surface(self.h, tris.ctypes.data_as(PI32), edges.ctypes.data_as(PI32), vb.ctypes.data_as(PI32))
        return tris, edges, vb

    def lumped_mass(self):
        m = np.zeros(self.n_soft_verts)
        lib().zref_lumped_mass(self.h, _pd(m))
        return m

    def affine_props(self):
        o = np.zeros((self.n_bodies - 0, 14))
        lib().zref_affine_props(self.h, _pd(o))
        return o

    # state
    def set_state(self, y, ydot, kappa=0.0, step=0):
        self._chk(lib().zref_set_state(self.h, _pd(_f64(y)), _pd(_f64(ydot)), float(kappa), int(step)))

    def get_state(self):
        y = np.zeros(self.n_dof); yd = np.zeros(self.n_dof); k = D(); st = I32()
        lib().zref_get_state(self.h, _pd(y), _pd(yd), C.byref(k), C.byref(st))
        return y, yd, k.value, st.value

    def set_kappa(self, kappa):
        self._chk(lib().zref_set_kappa(self.h, float(kappa)))

    def surface_positions(self, y):
        xs = np.zeros((self.n_surf, 3))
        lib().zref_surface_positions(self.h, _pd(_f64(y)), _pd(xs))
        return xs

    def candidates(self, xs0, xs1=None, r=None):
        r = self.params.dhat if r is None else r
        xs0 = _f64(xs0); xs1 = _f64(xs1) if xs1 is not None else None
        npt = I64(); nee = I64()
        cap = 1
        while True:
            pt = np.zeros((cap, 2), dtype=np.int32); ee = np.zeros((cap, 2), dtype=np.int32)
            rc = lib().zref_candidates(self.h, _pd(xs0), _pd(xs1), float(r), pt.ctypes.data_as(PI32), cap,
                                       C.byref(npt), ee.ctypes.data_as(PI32), cap, C.byref(nee))
            if rc == -4:
                cap = max(npt.value, nee.value, 1)
                continue
            self._chk(rc)
            return pt[:npt.value].copy(), ee[:nee.value].copy()

    def ip_assemble(self, y, grad=True, hess=True, mask=0):
        """Energy terms [inertia, elastic, orth, kinematic, barrier, friction, total,
        min distance] at y (static candidates rebuilt at y); gradient of the terms in
        `mask` (bit k = term k; 0 = all); the Hessian is kept for hessian_matvec."""
        terms = np.zeros(8)
        g = np.zeros(self.n_dof)
        flags = (1 if grad else 0) | (2 if hess else 0) | ((int(mask) & 0x3f) << 8)
        rc = lib().zref_ip_assemble(self.h, _pd(_f64(y)), flags, _pd(terms), _pd(g))
        self._chk(rc)
        return terms, g

    def hessian_matvec(self, v):
        out = np.zeros(self.n_dof)
        self._chk(lib().zref_hessian_matvec(self.h, _pd(_f64(v)), _pd(out)))
        return out

    def pcg_solve(self, rhs, rtol=None, max_iter=0):
        rtol = self.params.pcg_rtol if rtol is None else rtol
        sol = np.zeros(self.n_dof); it = I32(); rr = D()
        rc = lib().zref_pcg_solve(self.h, _pd(_f64(rhs)), _pd(sol), float(rtol), int(max_iter), C.byref(it), C.byref(rr))
        self._chk(rc)
        return sol, it.value, rr.value

    def ccd_max_step(self, y, p):
        a = D()
        self._chk(lib().zref_ccd_max_step(self.h, _pd(_f64(y)), _pd(_f64(p)), C.byref(a)))
        return a.value

    def friction_table(self):
        n = I64()
        lib().zref_friction_count(self.h, C.byref(n))
        ids = np.zeros((n.value, 5), dtype=np.int32); vals = np.zeros((n.value, 8))
        lib().zref_friction_table(self.h, ids.ctypes.data_as(PI32), _pd(vals))
        return ids, vals

    def step(self, n=1):
        st = (StepStats * n)()
        rc = lib().zref_step(self.h, n, st)
        out = [{f[0]: getattr(s, f[0]) for f in StepStats._fields_} for s in st]
        if rc != 0:
            raise OracleError(rc, lib().zref_last_error(self.h).decode())
        return out

    def contact_forces(self, y):
        """Contact force (N) on every body at y: soft bodies first, then affine bodies."""
        nb = self.n_bodies
        f = np.zeros((nb, 3))
        rc = lib().zref_contact_forces(self.h, _pd(_f64(y)), _pd(f))
        if rc != 0:
            raise OracleError(rc, "contact forces")
        return f

    def set_drive_target(self, body, q):
        """Kinematic target (12 values) of driven affine body `body` for the following
        steps; None returns to the scheduled target."""
        qq = _f64(q) if q is not None else None
        rc = lib().zref_set_drive_target(self.h, int(body), _pd(qq))
        if rc != 0:
            raise OracleError(rc, "set_drive_target")

    def set_springs(self, sv, k, targets):
        """Springs on distinct surface vertices sv with stiffness k (N/m) towards
        targets [n][3]; empty arrays remove them."""
        sv = np.ascontiguousarray(sv, dtype=np.int32)
        k = _f64(k)
        t = _f64(targets).reshape(-1, 3)
        rc = lib().zref_set_springs(self.h, len(sv), sv.ctypes.data_as(PI32), _pd(k), _pd(t))
        if rc != 0:
            raise OracleError(rc, "set_springs")

    def set_prismatic_joints(self, pairs, axes, kappa):
        """Prismatic joints between affine bodies pairs [n][2] with axes [n][3] (first
        body's rest frame) and stiffness kappa [n]; empty arrays remove them."""
        pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        ax = _f64(axes).reshape(-1, 3)
        kk = _f64(kappa).reshape(-1)
        rc = lib().zref_set_prismatic_joints(self.h, len(pr), pr.ctypes.data_as(PI32), _pd(ax), _pd(kk))
        if rc != 0:
            raise OracleError(rc, "set_prismatic_joints")

    def kinematic_al(self, tol, max_updates=8):
        """Augmented Lagrangian updates of the kinematic multipliers; returns the
        current multipliers [n_affine][12]."""
        n_aff = self.n_bodies - self.n_soft_bodies
        lam = np.zeros((max(n_aff, 1), 12))
        rc = lib().zref_kinematic_al(self.h, float(tol), int(max_updates), _pd(lam))
        if rc != 0:
            raise OracleError(rc, "kinematic_al")
        return lam[:n_aff]

    def record(self, enable=True):
        lib().zref_record(self.h, 1 if enable else 0)

    def records(self):
        n = I64()
        lib().zref_record_count(self.h, C.byref(n))
        out = []
        for k in range(n.value):
            st = I32(); kl = D(); kk = D()
            yt = np.zeros(self.n_dof); ydt = np.zeros(self.n_dof); yk = np.zeros(self.n_dof)
            lib().zref_record_get(self.h, k, C.byref(st), C.byref(kl), C.byref(kk), _pd(yt), _pd(ydt), _pd(yk))
            out.append({"step": st.value, "kappa_lag": kl.value, "kappa": kk.value,
                        "y_t": yt, "ydot_t": ydt, "y_k": yk})
        return out

    def pair_energy(self, kind, x12, rest_len2=(1.0, 1.0), project=True, ftype=-1):
        """Barrier energy, gradient and (projected) Hessian of one pair at the scene's
        kappa; ftype >= 0 takes that feature type's squared distance instead of the
        closest feature's."""
        e = D(); g = np.zeros(12); H = np.zeros((12, 12))
        rl = _f64(rest_len2)
        self._chk(lib().zref_pair_energy_typed(self.h, kind, _pd(_f64(x12)), _pd(rl), int(ftype), C.byref(e), _pd(g),
                                               _pd(H), 1 if project else 0))
        return e.value, g, H

    def tet_energy(self, tet, x12, project=True):
        e = D(); g = np.zeros(12); H = np.zeros((12, 12))
        rc = lib().zref_tet_energy(self.h, tet, _pd(_f64(x12)), C.byref(e), _pd(g), _pd(H), 1 if project else 0)
        if rc == -2:
            return float("inf"), g, H
        self._chk(rc)
        return e.value, g, H
