"""Python binding of libzema.so (argument marshalling only).

Every computation runs in the HIP library; this module converts scene descriptions
to the C structs of include/zema.h and passes torch device tensors as raw pointers.
Importing it without the built library raises immediately: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libzema.so")

D, I32, I64 = C.c_double, C.c_int32, C.c_int64
PD, PI32, PI64 = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
VP = C.c_void_p

OK, E_ARG, E_MESH, E_INTERSECT, E_CAPACITY, E_NEWTON, E_LINESEARCH, E_PCG, E_NONFINITE, E_DEVICE = \
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9
GRAD, HESS, REBUILD, TERMS_SHIFT = 1, 2, 4, 8
TERM_NAMES = ("inertia", "elastic", "orthogonality", "kinematic", "barrier", "friction", "total", "min_distance")


class Params(C.Structure):
    _fields_ = [("dt", D), ("dhat", D), ("kappa", D), ("mu", D), ("eps_v", D), ("gravity", D * 3),
                ("newton_tol", D), ("pcg_rtol", D), ("ccd_s", D), ("newton_max", I32), ("pcg_max", I32),
                ("precision", I32), ("warm_start", I32)]


class SoftDesc(C.Structure):
    _fields_ = [("n_verts", I32), ("n_tets", I32), ("rest_pos", PD), ("tets", PI32), ("pos0", PD), ("vel0", PD),
                ("E", D), ("nu", D), ("rho", D), ("model", I32), ("pad_", I32), ("tris", PI32), ("n_tris", I32),
                ("pad2_", I32)]


class AffineDesc(C.Structure):
    _fields_ = [("n_verts", I32), ("n_tris", I32), ("rest_pos", PD), ("tris", PI32), ("rho", D),
                ("stiffness", D), ("qdot0", D * 12), ("mode", I32), ("pad_", I32), ("kappa_A", D),
                ("target_vel", D * 3), ("target_stop", D)]


class GraspParams(C.Structure):
    _fields_ = [("k", D), ("f_star", D), ("max_close_steps", I32), ("lift_steps", I32), ("shake_steps", I32),
                ("object_body", I32), ("lift_speed", D), ("shake_amplitude", D), ("shake_frequency", D),
                ("shake_axis", D * 3), ("ground_body", I32), ("pad_", I32)]


class GraspResult(C.Structure):
    _fields_ = [("status", I32), ("close_steps", I32), ("total_steps", I32), ("success", I32), ("n_fingers", I32),
                ("pad_", I32), ("ground_force", D), ("finger_force_max", D)]


class StepStats(C.Structure):
    _fields_ = [("status", I32), ("newton_iters", I32), ("pcg_iters", I32), ("ls_backtracks", I32),
                ("n_pt_active", I32), ("n_ee_active", I32), ("n_pt_cand", I32), ("n_ee_cand", I32),
                ("warm_learned", I32), ("pcg_breakdowns", I32), ("al_updates", I32), ("pad_", I32),
                ("alpha_ccd_min", D), ("kappa", D), ("d_min", D), ("energy", D), ("ms_total", D),
                ("ms_assemble", D), ("ms_pcg", D), ("ms_broad", D), ("ms_ccd", D), ("ms_linesearch", D),
                ("ms_warm", D)]


_LIB = None

# (name, argtypes) of every entry point of include/zema.h
SIGNATURES = [
    ("zema_scene_create", [C.POINTER(Params), C.POINTER(SoftDesc), I32, C.POINTER(AffineDesc), I32, VP,
                           C.POINTER(VP)]),
    ("zema_scene_destroy", [VP]),
    ("zema_contact_forces", [VP, VP, PD]),
    ("zema_set_drive_target", [VP, I32, PD]),
    ("zema_set_springs", [VP, I32, PI32, PD, PD]),
    ("zema_kinematic_al", [VP, D, I32, PD]),
    ("zema_set_prismatic_joints", [VP, I32, PI32, PD, PD]),
    ("zema_grasp_run", [VP, C.POINTER(GraspParams), C.POINTER(GraspResult), PD, I32]),
    ("zema_status_string", [C.c_int]),
    ("zema_last_error", [VP]),
    ("zema_sizes", [VP, PI64]),
    ("zema_set_state", [VP, VP, VP, D, I32]),
    ("zema_get_state", [VP, VP, VP, PD, PI32]),
    ("zema_set_kappa", [VP, D]),
    ("zema_surface_positions", [VP, VP, VP]),
    ("zema_contact_candidates", [VP, VP, VP, D, VP, I64, PI64, VP, I64, PI64]),
    ("zema_ip_assemble", [VP, VP, C.c_uint32, PD, VP]),
    ("zema_hessian_matvec", [VP, VP, VP]),
    ("zema_hessian_bsr", [VP, VP, VP, VP, I64, PI64]),
    ("zema_surface_view", [VP, VP, VP, VP, VP]),
    ("zema_pcg_solve", [VP, VP, VP, D, I32, PI32, PD]),
    ("zema_ccd_max_step", [VP, VP, VP, PD]),
    ("zema_step", [VP, I32, C.POINTER(StepStats)]),
    ("zema_friction_table", [VP, PI64, PI32, PD, I64]),
    ("zema_intersection_count", [VP, VP, PI64, PI64, PI64, VP, I64]),
    ("zema_kernel_timer", [VP, I32, I32]),
    ("zema_kernel_time", [VP, I32, PD, PI64, PD]),
    ("zema_mlp_create", [VP, C.POINTER(VP)]),
    ("zema_mlp_destroy", [VP]),
    ("zema_mlp_last_error", [VP]),
    ("zema_mlp_set_weights", [VP, C.POINTER(C.c_float)]),
    ("zema_mlp_get_weights", [VP, C.POINTER(C.c_float)]),
    ("zema_mlp_forward", [VP, VP, I64, VP]),
    ("zema_mlp_grad", [VP, VP, VP, I64, VP, PD]),
    ("zema_mlp_grad_noalloc", [VP, VP, VP, I64, VP, PD]),
    ("zema_mlp_train_step", [VP, VP, VP, I64, VP, I64, C.c_float, PD]),
    ("zema_batch_create", [VP, I32, VP, PI32, VP, PI32, VP, C.POINTER(VP)]),
    ("zema_batch_layout", [VP, C.POINTER(I32), PI64]),
    ("zema_tune", [VP, I32, I32]),
    ("zema_step_group", [C.POINTER(VP), I32, I32, C.POINTER(VP), PI32]),
    ("zema_tune_get", [VP, I32, PI32]),
    ("zema_autotune", [VP, PI32, PI32, PD]),
    ("zema_scene_set_mlp", [VP, VP]),
    ("zema_scene_features", [VP, VP]),
    ("zema_scene_warm_target", [VP, VP]),
    ("zema_warm_fit", [VP, I32, VP, VP]),
]
MLP_PARAMS = 9603
MLP_FEATURES = 16
WARM_EXPLICIT, WARM_LEARNED = 0, 1
(TUNE_PCG_GRAPH, TUNE_SPMV_LANES, TUNE_UPDATE_BLOCK, TUNE_PCG_FORM, TUNE_BATCH_ASYNC, TUNE_CG_ROWS,
 TUNE_WARM_FIT) = 0, 1, 2, 3, 4, 5, 6
KT_SPMV, KT_TET, KT_CONTACT, KT_QUERY, KT_CCD = range(5)


def lib():
    """Load libzema.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2311_05945_amd/build.py; "
                               "there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        for name, args in SIGNATURES:
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.zema_scene_destroy.restype = None
        L.zema_mlp_destroy.restype = None
        L.zema_status_string.restype = C.c_char_p
        L.zema_last_error.restype = C.c_char_p
        L.zema_mlp_last_error.restype = C.c_char_p
        _LIB = L
    return _LIB


class ZemaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"zema status {code}: {msg}")
        self.code = code


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _pd(a):
    return None if a is None else a.ctypes.data_as(PD)


def _ptr(t):
    """Raw device pointer of a torch tensor (None for None)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def params_struct(p) -> Params:
    return Params(p.dt, p.dhat, p.kappa, p.mu, p.eps_v, (D * 3)(*p.gravity), p.newton_tol, p.pcg_rtol, p.ccd_s,
                  p.newton_max, p.pcg_max, p.precision, p.warm_start)


class Scene:
    """A scene of libzema bound to one torch (HIP) stream."""

    def __init__(self, scene, device="cuda:0", stream=None, _batch=None):
        """One scene (a `scenegen.Scene`), or with `_batch` a list of scenes stepped
        together (see `Scene.batch`)."""
        import torch
        self.torch = torch
        self.device = torch.device(device)
        L = lib()
        self._keep = []
        scenes = _batch if _batch is not None else [scene]
        all_softs = [b for sc in scenes for b in sc.softs]
        all_affs = [b for sc in scenes for b in sc.affines]
        self.n_driven = sum(1 for b in all_affs if b.mode == 2)
        self.n_soft_bodies = len(all_softs)
        softs = (SoftDesc * max(1, len(all_softs)))()
        for k, b in enumerate(all_softs):
            rp = _f64(b.rest_pos); tt = np.ascontiguousarray(b.tets, dtype=np.int32)
            p0 = _f64(b.pos0) if b.pos0 is not None else None
            v0 = _f64(b.vel0) if b.vel0 is not None else None
            tr = getattr(b, "tris", None)
            tr = np.ascontiguousarray(tr, dtype=np.int32).reshape(-1, 3) if tr is not None else None
            self._keep += [rp, tt, p0, v0, tr]
            softs[k] = SoftDesc(len(rp), len(tt), _pd(rp), tt.ctypes.data_as(PI32), _pd(p0), _pd(v0), b.E, b.nu, b.rho,
                                getattr(b, "model", 0), 0, tr.ctypes.data_as(PI32) if tr is not None else None,
                                len(tr) if tr is not None else 0, 0)
        affs = (AffineDesc * max(1, len(all_affs)))()
        for k, b in enumerate(all_affs):
            rp = _f64(b.rest_pos); tt = np.ascontiguousarray(b.tris, dtype=np.int32)
            self._keep += [rp, tt]
            affs[k] = AffineDesc(len(rp), len(tt), _pd(rp), tt.ctypes.data_as(PI32), b.rho, b.stiffness,
                                 (D * 12)(*np.asarray(b.qdot0, dtype=float)), b.mode, 0, b.kappa_A,
                                 (D * 3)(*np.asarray(b.target_vel, dtype=float)), b.target_stop)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            if _batch is None:
                P = params_struct(scene.params)
                rc = L.zema_scene_create(C.byref(P), softs, len(all_softs), affs, len(all_affs),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h))
            else:
                ns = len(scenes)
                Ps = (Params * ns)(*[params_struct(sc.params) for sc in scenes])
                so = np.cumsum([0] + [len(sc.softs) for sc in scenes]).astype(np.int32)
                ao = np.cumsum([0] + [len(sc.affines) for sc in scenes]).astype(np.int32)
                self._keep += [so, ao]
                rc = L.zema_batch_create(Ps, ns, softs, so.ctypes.data_as(PI32), affs, ao.ctypes.data_as(PI32),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != 0:
            raise ZemaError(rc, L.zema_status_string(rc).decode())
        self.h = h
        s = np.zeros(8, dtype=np.int64)
        L.zema_sizes(self.h, s.ctypes.data_as(PI64))
        (self.n_dof, self.n_soft_verts, self.n_tets, self.n_surf, self.n_tris, self.n_edges,
         self.n_free_bodies, self.n_bodies) = [int(x) for x in s]
        ns = I32()
        L.zema_batch_layout(self.h, C.byref(ns), None)
        self.n_scenes = ns.value
        self.layout = np.zeros((self.n_scenes, 8), dtype=np.int64)
        L.zema_batch_layout(self.h, C.byref(ns), self.layout.ctypes.data_as(PI64))
        self.params = scenes[0].params

    @classmethod
    def batch(cls, scenes, device="cuda:0", stream=None):
        """Scenes stepped together: one launch per phase over all of them."""
        return cls(None, device, stream, _batch=list(scenes))

    def scene_dofs(self, k):
        """DOF indices of scene k of a batch in the concatenated y."""
        v0, v1, f0, f1 = (int(x) for x in self.layout[k, :4])
        n3 = 3 * self.n_soft_verts
        return np.concatenate([np.arange(3 * v0, 3 * v1), np.arange(n3 + 12 * f0, n3 + 12 * f1)])

    def __del__(self):
        if getattr(self, "h", None):
            try:
                lib().zema_scene_destroy(self.h)
            except Exception:  # interpreter shutdown: module globals already gone
                pass
            self.h = None

    def _chk(self, rc):
        if rc != 0:
            raise ZemaError(rc, lib().zema_last_error(self.h).decode())

    def _dev(self, a, dtype=None):
        t = self.torch
        dtype = dtype or t.float64
        if isinstance(a, t.Tensor):
            return a.to(device=self.device, dtype=dtype).contiguous()
        return t.as_tensor(np.asarray(a), dtype=dtype, device=self.device).contiguous()

    def zeros(self, *shape, dtype=None):
        return self.torch.zeros(*shape, dtype=dtype or self.torch.float64, device=self.device)

    # ---- state
    def set_state(self, y, ydot, kappa=0.0, step=0):
        y = self._dev(y); yd = self._dev(ydot)
        self._chk(lib().zema_set_state(self.h, _ptr(y), _ptr(yd), float(kappa), int(step)))

    def get_state(self):
        y = self.zeros(self.n_dof); yd = self.zeros(self.n_dof); k = D(); st = I32()
        self._chk(lib().zema_get_state(self.h, _ptr(y), _ptr(yd), C.byref(k), C.byref(st)))
        return y, yd, k.value, st.value

    def set_kappa(self, kappa):
        self._chk(lib().zema_set_kappa(self.h, float(kappa)))

    def surface_positions(self, y):
        y = self._dev(y)
        xs = self.zeros(self.n_surf, 3)
        self._chk(lib().zema_surface_positions(self.h, _ptr(y), _ptr(xs)))
        return xs

    # ---- hot path
    def contact_candidates(self, xs0, xs1=None, r=None):
        r = self.params.dhat if r is None else r
        xs0 = self._dev(xs0); xs1 = self._dev(xs1) if xs1 is not None else None
        npt, nee = I64(), I64()
        cap = 1024
        while True:
            pt = self.torch.zeros((cap, 2), dtype=self.torch.int32, device=self.device)
            ee = self.torch.zeros((cap, 2), dtype=self.torch.int32, device=self.device)
            rc = lib().zema_contact_candidates(self.h, _ptr(xs0), _ptr(xs1), float(r), _ptr(pt), cap,
                                               C.byref(npt), _ptr(ee), cap, C.byref(nee))
            if rc == E_CAPACITY:
                cap = max(npt.value, nee.value, 1)
                continue
            self._chk(rc)
            return pt[:npt.value], ee[:nee.value]

    def ip_assemble(self, y, grad=True, hess=True, mask=0, rebuild=True):
        """Energy terms and gradient at y; rebuild=False evaluates on the stored
        candidate set instead of rebuilding it statically at y."""
        y = self._dev(y)
        terms = np.zeros(8)
        g = self.zeros(self.n_dof) if grad else None
        flags = ((GRAD if grad else 0) | (HESS if hess else 0) | (REBUILD if rebuild else 0)
                 | ((int(mask) & 0x3F) << TERMS_SHIFT))
        self._chk(lib().zema_ip_assemble(self.h, _ptr(y), flags, _pd(terms), _ptr(g)))
        return terms, g

    def hessian_matvec(self, v):
        v = self._dev(v)
        out = self.zeros(self.n_dof)
        self._chk(lib().zema_hessian_matvec(self.h, _ptr(v), _ptr(out)))
        return out

    def hessian_bsr(self):
        """(row_ptr [n_dof/3 + 1], col [nnzb], val [nnzb][3][3]) device tensors of the
        last assembled Hessian."""
        t = self.torch
        n = I64()
        rc = lib().zema_hessian_bsr(self.h, None, None, None, 0, C.byref(n))
        if rc not in (OK, E_CAPACITY):
            self._chk(rc)
        rp = t.zeros(self.n_dof // 3 + 1, dtype=t.int32, device=self.device)
        col = t.zeros(max(n.value, 1), dtype=t.int32, device=self.device)
        val = t.zeros((max(n.value, 1), 3, 3), dtype=t.float64, device=self.device)
        self._chk(lib().zema_hessian_bsr(self.h, _ptr(rp), _ptr(col), _ptr(val), n.value, C.byref(n)))
        return rp, col[:n.value], val[:n.value]

    def surface_view(self):
        """(tris [n_tris][3], edges [n_edges][2], vbody [n_surf], vsrc [n_surf]) device
        tensors: the topology the candidate pair ids index."""
        t = self.torch
        tris = t.zeros((max(self.n_tris, 1), 3), dtype=t.int32, device=self.device)
        edges = t.zeros((max(self.n_edges, 1), 2), dtype=t.int32, device=self.device)
        vb = t.zeros(max(self.n_surf, 1), dtype=t.int32, device=self.device)
        vs = t.zeros(max(self.n_surf, 1), dtype=t.int32, device=self.device)
        self._chk(lib().zema_surface_view(self.h, _ptr(tris), _ptr(edges), _ptr(vb), _ptr(vs)))
        return tris[:self.n_tris], edges[:self.n_edges], vb[:self.n_surf], vs[:self.n_surf]

    def pcg_solve(self, rhs, rtol=None, max_iter=0):
        rtol = self.params.pcg_rtol if rtol is None else rtol
        rhs = self._dev(rhs)
        sol = self.zeros(self.n_dof); it = I32(); rr = D()
        self._chk(lib().zema_pcg_solve(self.h, _ptr(rhs), _ptr(sol), float(rtol), int(max_iter), C.byref(it),
                                       C.byref(rr)))
        return sol, it.value, rr.value

    def ccd_max_step(self, y, p):
        y = self._dev(y); p = self._dev(p)
        a = D()
        self._chk(lib().zema_ccd_max_step(self.h, _ptr(y), _ptr(p), C.byref(a)))
        return a.value

    def step(self, n=1):
        """Statistics of n steps: a list of n dicts (single scene) or of n * n_scenes
        dicts, step-major (batch)."""
        m = n * self.n_scenes
        st = (StepStats * max(m, 1))()
        rc = lib().zema_step(self.h, n, st)
        out = [{f[0]: getattr(s, f[0]) for f in StepStats._fields_} for s in st[:m]]
        if rc != 0:
            raise ZemaError(rc, lib().zema_last_error(self.h).decode())
        return out

    def friction_table(self):
        n = I64()
        cap = 0
        while True:
            ids = np.zeros((max(cap, 1), 5), dtype=np.int32); vals = np.zeros((max(cap, 1), 8))
            rc = lib().zema_friction_table(self.h, C.byref(n), ids.ctypes.data_as(PI32), _pd(vals), cap)
            if rc == E_CAPACITY:
                cap = n.value
                continue
            self._chk(rc)
            return ids[:n.value], vals[:n.value]


    def contact_forces(self, y):
        """zema_contact_forces: contact force (N) on every body at y (host [n_bodies][3],
        soft bodies first)."""
        y = self._dev(y)
        f = np.zeros((self.n_bodies, 3))
        self._chk(lib().zema_contact_forces(self.h, _ptr(y), _pd(f)))
        return f

    def set_drive_target(self, body, q):
        """zema_set_drive_target: kinematic target (12 values) of driven affine body
        `body`; None returns to the scheduled target."""
        qq = np.ascontiguousarray(q, dtype=np.float64) if q is not None else None
        self._chk(lib().zema_set_drive_target(self.h, int(body), _pd(qq)))

    def set_springs(self, sv, k, targets):
        """zema_set_springs: springs on distinct surface vertices sv (stiffness k N/m)
        towards targets [n][3]; empty arrays remove them."""
        sv = np.ascontiguousarray(sv, dtype=np.int32)
        kk = np.ascontiguousarray(k, dtype=np.float64)
        t = np.ascontiguousarray(targets, dtype=np.float64).reshape(-1, 3)
        self._chk(lib().zema_set_springs(self.h, len(sv), sv.ctypes.data_as(PI32), _pd(kk), _pd(t)))

    def set_prismatic_joints(self, pairs, axes, kappa):
        """zema_set_prismatic_joints: joints between affine bodies pairs [n][2] with axes
        [n][3] (first body's rest frame) and stiffness kappa [n]."""
        pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        ax = np.ascontiguousarray(axes, dtype=np.float64).reshape(-1, 3)
        kk = np.ascontiguousarray(kappa, dtype=np.float64).reshape(-1)
        self._chk(lib().zema_set_prismatic_joints(self.h, len(pr), pr.ctypes.data_as(PI32), _pd(ax), _pd(kk)))

    def kinematic_al(self, tol, max_updates=8):
        """zema_kinematic_al: multiplier updates of the kinematic energy; returns the
        multipliers [n_affine][12]."""
        n_aff = self.n_bodies - self.n_soft_bodies
        lam = np.zeros((max(n_aff, 1), 12))
        self._chk(lib().zema_kinematic_al(self.h, float(tol), int(max_updates), _pd(lam)))
        return lam[:n_aff]

    def grasp_run(self, k=20.0, f_star=0.5, max_close_steps=200, lift_steps=100, lift_speed=0.1,
                  shake_steps=0, shake_amplitude=0.0, shake_frequency=0.0, shake_axis=(1.0, 0.0, 0.0),
                  object_body=0, ground_body=-1, trace_cap=4096):
        """zema_grasp_run: AutoGrasp, Lift and Shake; returns (result dict, trace rows
        [phase, |f_ground|, |f_finger| ...] per step)."""
        gp = GraspParams(k, f_star, max_close_steps, lift_steps, shake_steps, object_body, lift_speed,
                         shake_amplitude, shake_frequency, (D * 3)(*shake_axis), ground_body, 0)
        res = GraspResult()
        trace = np.zeros((max(trace_cap, 1), 2 + self.n_driven))
        rc = lib().zema_grasp_run(self.h, C.byref(gp), C.byref(res), _pd(trace), trace_cap)
        out = {f[0]: getattr(res, f[0]) for f in GraspResult._fields_ if f[0] != "pad_"}
        if rc != 0:
            raise ZemaError(rc, lib().zema_last_error(self.h).decode())
        return out, trace[:min(res.total_steps, trace_cap), :2 + res.n_fingers]

    def intersection_count(self, y, cap=1024):
        """(intersecting edge-triangle pairs, inverted tets, uncertain, uncertain pairs)."""
        y = self._dev(y)
        ni, nv, nu = I64(), I64(), I64()
        unc = self.torch.zeros((max(cap, 1), 2), dtype=self.torch.int32, device=self.device)
        self._chk(lib().zema_intersection_count(self.h, _ptr(y), C.byref(ni), C.byref(nv), C.byref(nu), _ptr(unc),
                                                cap))
        return ni.value, nv.value, nu.value, unc[:min(nu.value, cap)]

    def tune(self, knob, value):
        self._chk(lib().zema_tune(self.h, int(knob), int(value)))

    def tune_get(self, knob):
        v = I32()
        self._chk(lib().zema_tune_get(self.h, int(knob), C.byref(v)))
        return v.value

    def spmv_lanes(self):
        """Lanes per soft row of the PCG kernels (after the two-launch form's fallback)."""
        lanes = self.tune_get(TUNE_SPMV_LANES)
        return 8 if lanes == 4 and self.tune_get(TUNE_PCG_FORM) == 0 else lanes

    def autotune(self):
        """(lanes per soft row, update block, microseconds per PCG iteration) chosen."""
        l, u, t = I32(), I32(), D()
        self._chk(lib().zema_autotune(self.h, C.byref(l), C.byref(u), C.byref(t)))
        return l.value, u.value, t.value

    def kernel_timer(self, group, enable=True):
        self._chk(lib().zema_kernel_timer(self.h, int(group), 1 if enable else 0))

    def kernel_time(self, group):
        """(total ms, launches, algorithmic bytes) of a timed kernel group."""
        ms = D(); n = I64(); b = D()
        self._chk(lib().zema_kernel_time(self.h, int(group), C.byref(ms), C.byref(n), C.byref(b)))
        return ms.value, n.value, b.value


    # ---- learned initial guess
    def set_mlp(self, mlp):
        self._mlp = mlp                      # keep the network alive while attached
        self._chk(lib().zema_scene_set_mlp(self.h, mlp.h if mlp is not None else None))

    def features(self):
        f = self.torch.zeros((self.n_soft_verts, MLP_FEATURES), dtype=self.torch.float32, device=self.device)
        self._chk(lib().zema_scene_features(self.h, _ptr(f)))
        return f

    def warm_target(self):
        t = self.torch.zeros((self.n_soft_verts, 3), dtype=self.torch.float32, device=self.device)
        self._chk(lib().zema_scene_warm_target(self.h, _ptr(t)))
        return t

    def warm_fit(self, corr, mode):
        """The learned guess's per-soft-body fit (0 copy, 1 affine, 2 mean) of a
        correction field [n_soft_verts][3] at the current state."""
        c = self._dev(corr, self.torch.float32).reshape(self.n_soft_verts, 3).contiguous()
        out = self.torch.empty_like(c)
        self._chk(lib().zema_warm_fit(self.h, int(mode), _ptr(c), _ptr(out)))
        return out


class Mlp:
    """The warm-start network of libzema (weights on the device, FP32 master copy)."""

    def __init__(self, theta=None, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            rc = lib().zema_mlp_create(C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != 0:
            raise ZemaError(rc, lib().zema_status_string(rc).decode())
        self.h = h
        if theta is not None:
            self.set_weights(theta)

    def __del__(self):
        if getattr(self, "h", None):
            try:
                lib().zema_mlp_destroy(self.h)
            except Exception:
                pass
            self.h = None

    def _chk(self, rc):
        if rc != 0:
            raise ZemaError(rc, lib().zema_mlp_last_error(self.h).decode())

    def _dev32(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device=self.device, dtype=t.float32).contiguous()
        return t.as_tensor(np.asarray(a), dtype=t.float32, device=self.device).contiguous()

    def set_weights(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        if th.shape != (MLP_PARAMS,):
            raise ValueError(f"expected {MLP_PARAMS} parameters")
        self._chk(lib().zema_mlp_set_weights(self.h, th.ctypes.data_as(C.POINTER(C.c_float))))

    def get_weights(self):
        th = np.zeros(MLP_PARAMS, dtype=np.float32)
        self._chk(lib().zema_mlp_get_weights(self.h, th.ctypes.data_as(C.POINTER(C.c_float))))
        return th

    def forward(self, feat):
        f = self._dev32(feat)
        out = self.torch.zeros((f.shape[0], 3), dtype=self.torch.float32, device=self.device)
        self._chk(lib().zema_mlp_forward(self.h, _ptr(f), f.shape[0], _ptr(out)))
        return out

    def grad(self, feat, target):
        f = self._dev32(feat); t = self._dev32(target)
        g = self.torch.zeros(MLP_PARAMS, dtype=self.torch.float32, device=self.device)
        loss = D()
        self._chk(lib().zema_mlp_grad(self.h, _ptr(f), _ptr(t), f.shape[0], _ptr(g), C.byref(loss)))
        return loss.value, g

    def grad_noalloc(self, feat, target, grad):
        """zema_mlp_grad_noalloc: loss and gradient into the caller's grad (device FP32
        [MLP_PARAMS]); feat [n][16] and target [n][3] are device FP32, contiguous.  The
        library allocates no device memory for the call."""
        for t, shape in ((feat, (feat.shape[0], 16)), (target, (feat.shape[0], 3)), (grad, (MLP_PARAMS,))):
            if t.dtype != self.torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
                raise ValueError(f"grad_noalloc needs contiguous device float32 tensors of shape {shape}")
        loss = D()
        self._chk(lib().zema_mlp_grad_noalloc(self.h, _ptr(feat), _ptr(target), feat.shape[0], _ptr(grad),
                                              C.byref(loss)))
        return loss.value

    def train_step(self, feat, target, idx, lr):
        """One Adam step on rows idx (device int32 tensor) of feat / target (device)."""
        loss = D()
        self._chk(lib().zema_mlp_train_step(self.h, _ptr(feat), _ptr(target), feat.shape[0], _ptr(idx),
                                            idx.shape[0], float(lr), C.byref(loss)))
        return loss.value


def scene_create(scene, device="cuda:0", stream=None) -> Scene:
    return Scene(scene, device, stream)


def step_group(objs, n=1):
    """zema_step_group: steps the scene objects `objs` (single scenes or batches, each
    created on its own stream) concurrently, n steps each; returns one statistics list
    per object (as Scene.step)."""
    k = len(objs)
    arrs = [(StepStats * max(n * o.n_scenes, 1))() for o in objs]
    hs = (VP * k)(*[o.h for o in objs])
    ps = (VP * k)(*[C.cast(a, VP) for a in arrs])
    status = (I32 * k)()
    rc = lib().zema_step_group(hs, k, n, ps, status)
    outs = [[{f[0]: getattr(s, f[0]) for f in StepStats._fields_} for s in a[:n * o.n_scenes]]
            for a, o in zip(arrs, objs)]
    if rc != 0:
        bad = next(i for i in range(k) if status[i] != 0)
        raise ZemaError(rc, lib().zema_last_error(objs[bad].h).decode())
    return outs


def batch_group(scenes, n_groups=4, device="cuda:0"):
    """The scenes split into n_groups batch objects of similar size (by soft vertex
    count, largest first, dealt round-robin), each on a stream of its own; step them
    with step_group."""
    import torch
    order = sorted(range(len(scenes)), key=lambda i: -sum(len(b.rest_pos) for b in scenes[i].softs))
    groups = [order[g::n_groups] for g in range(n_groups) if order[g::n_groups]]
    objs = [Scene.batch([scenes[i] for i in g], device=device, stream=torch.cuda.Stream(device=device))
            for g in groups]
    return objs, groups
