"""Thin ctypes binding of libbdem.so (include/bdem.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides the device workspace (a uint8 tensor) and the stream.  There
is no CPU fallback: if the library is missing or cannot be loaded, importing
this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

import torch  # loads the HIP runtime the library binds to

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbdem.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2308_10459_amd.build`")
_lib = C.CDLL(LIB_PATH)

BDEM_OK, BDEM_W_NOT_CONVERGED, BDEM_W_LS_FAILED = 0, 1, 2
BDEM_E_INVALID, BDEM_E_HIP, BDEM_E_NOMEM, BDEM_E_NONFINITE = -1, -2, -3, -4
BDEM_E_DEGENERATE, BDEM_E_STATE, BDEM_E_CAPACITY = -5, -6, -7
BDEM_FREE, BDEM_FIXED, BDEM_KINEMATIC = 0, 1, 2
BDEM_PREC_FP64, BDEM_PREC_MIXED = 0, 1
BDEM_SOLVER_NEWTON, BDEM_SOLVER_FIRST_ORDER = 0, 1
BDEM_INTEGRATOR_EULER, BDEM_INTEGRATOR_MIDPOINT = 0, 1
BDEM_PRECOND_BLOCK_JACOBI, BDEM_PRECOND_AMG = 0, 1
BDEM_EGH_E, BDEM_EGH_G, BDEM_EGH_H, BDEM_EGH_PSD, BDEM_EGH_POTENTIAL_ONLY = 1, 2, 4, 8, 16
BDEM_EGH_GN, BDEM_EGH_PCG_MATRIX = 32, 64
BDEM_SCRATCH_BYTES = 64 << 20
BDEM_HESS_EIGEN_CLAMP, BDEM_HESS_GAUSS_NEWTON = 0, 1

_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_u8p = C.POINTER(C.c_uint8)
_i64p = C.POINTER(C.c_int64)


class bdem_particles(C.Structure):
    _fields_ = [("n", C.c_int32), ("pos", _dp), ("quat", _dp), ("vel", _dp), ("qvel", _dp),
                ("radius", _dp), ("material", _i32p), ("flags", _u8p), ("scene", _i32p)]


class bdem_bonds(C.Structure):
    _fields_ = [("nb", C.c_int64), ("ij", _i32p), ("material", _i32p)]


class bdem_material(C.Structure):
    _fields_ = [("young", C.c_double), ("poisson", C.c_double), ("density", C.c_double),
                ("sigma_c", C.c_double), ("tau_c", C.c_double), ("stiff_scale", C.c_double * 4),
                ("shear_mode", C.c_int32), ("tension_only", C.c_int32)]


class bdem_options(C.Structure):
    _fields_ = [("gravity", C.c_double * 3), ("ground_normal", C.c_double * 3),
                ("ground_offset", C.c_double), ("k_contact", C.c_double), ("mu_s", C.c_double),
                ("mu_r", C.c_double), ("k_self", C.c_double), ("contact_margin", C.c_double),
                ("newton_tol", C.c_double), ("newton_rtol", C.c_double),
                ("armijo_c", C.c_double), ("cg_rtol_max", C.c_double), ("max_newton", C.c_int32),
                ("max_cg", C.c_int32), ("max_ls", C.c_int32), ("precision", C.c_int32),
                ("break_each_step", C.c_int32), ("cg_chunk", C.c_int32), ("use_graph", C.c_int32),
                ("solver", C.c_int32), ("integrator", C.c_int32), ("preconditioner", C.c_int32),
                ("hessian", C.c_int32), ("amg_refresh", C.c_int32)]


class bdem_step_stats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("cg_iters", C.c_int32), ("ls_backtracks", C.c_int32),
                ("status", C.c_int32), ("bonds_broken", C.c_int64), ("grad0", C.c_double),
                ("grad_final", C.c_double), ("phi", C.c_double), ("t_ms", C.c_double * 8)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "t_ms"}
        d["t_ms"] = list(self.t_ms)
        return d


class bdem_tuning(C.Structure):
    _fields_ = [("spmv_threads", C.c_int32), ("spmv_trips", C.c_int32), ("update_rows", C.c_int32),
                ("cg_chunk", C.c_int32), ("use_graph", C.c_int32), ("pad_", C.c_int32),
                ("spmv_us", C.c_double), ("update_us", C.c_double), ("pcg_us_per_iter", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


_ctx_p = C.c_void_p
_sig = {
    "bdem_default_options": (None, [C.POINTER(bdem_options)]),
    "bdem_workspace_bytes": (C.c_size_t, [C.POINTER(bdem_particles), C.POINTER(bdem_bonds),
                                          C.POINTER(bdem_options)]),
    "bdem_create": (C.c_int, [C.POINTER(bdem_particles), C.POINTER(bdem_bonds),
                              C.POINTER(bdem_material), C.c_int32, C.POINTER(bdem_options),
                              C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(_ctx_p)]),
    "bdem_create_in_scratch": (C.c_int, [C.POINTER(bdem_particles), C.POINTER(bdem_bonds),
                                         C.POINTER(bdem_material), C.c_int32, C.POINTER(bdem_options),
                                         C.c_void_p, C.POINTER(_ctx_p)]),
    "bdem_step": (C.c_int, [_ctx_p, C.c_double, C.POINTER(bdem_step_stats)]),
    "bdem_step_batched": (C.c_int, [_ctx_p, _dp, C.POINTER(bdem_step_stats)]),
    "bdem_energy_grad_hess": (C.c_int, [_ctx_p, C.c_double, C.c_int32, _dp, _dp, _dp, _dp,
                                        _dp, _dp]),
    "bdem_break_bonds": (C.c_int, [_ctx_p, _i64p, _u8p]),
    "bdem_contact_pairs": (C.c_int, [_ctx_p, C.c_int64, _i32p, _i64p]),
    "bdem_precond_apply": (C.c_int, [_ctx_p, C.c_double, _dp, _dp, _dp, _dp]),
    "bdem_hess_apply": (C.c_int, [_ctx_p, C.c_double, _dp, _dp, _dp, _dp]),
    "bdem_get_state": (C.c_int, [_ctx_p, _dp, _dp, _dp, _dp, _u8p]),
    "bdem_set_state": (C.c_int, [_ctx_p, _dp, _dp, _dp, _dp, _u8p]),
    "bdem_sizes": (C.c_int, [_ctx_p, _i32p, _i64p, _i32p]),
    "bdem_set_profiling": (C.c_int, [_ctx_p, C.c_int32]),
    "bdem_profile_counts": (C.c_int, [_ctx_p, _i32p, _i32p]),
    "bdem_autotune": (C.c_int, [_ctx_p, _dp, C.POINTER(bdem_tuning)]),
    "bdem_get_tuning": (C.c_int, [_ctx_p, C.POINTER(bdem_tuning)]),
    "bdem_set_tuning": (C.c_int, [_ctx_p, C.POINTER(bdem_tuning)]),
    "bdem_destroy": (None, [_ctx_p]),
    "bdem_last_error": (C.c_char_p, [_ctx_p]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class BdemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bdem error {code}: {msg}")
        self.code = code


def _p(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# same-named wrappers of the C entry points
# ---------------------------------------------------------------------------

def bdem_default_options(**overrides):
    o = bdem_options()
    _lib.bdem_default_options(C.byref(o))
    for k, v in overrides.items():
        if k in ("gravity", "ground_normal"):
            getattr(o, k)[:] = list(v)
        else:
            setattr(o, k, v)
    return o


def bdem_last_error(ctx=None):
    m = _lib.bdem_last_error(ctx)
    return m.decode() if m else ""


def _check(rc, ctx=None):
    if rc < 0:
        raise BdemError(rc, bdem_last_error(ctx))
    return rc


class _Inputs:
    """Keeps the numpy arrays behind the C structs alive."""

    def __init__(self, scene):
        self.pos = _f64(scene.pos)
        self.quat = _f64(scene.quat)
        self.vel = _f64(scene.vel)
        self.qvel = _f64(scene.qvel)
        self.radius = _f64(scene.radius)
        self.pmat = np.ascontiguousarray(scene.pmat, dtype=np.int32)
        self.flags = np.ascontiguousarray(scene.flags, dtype=np.uint8)
        self.sid = None if scene.scene_id is None else np.ascontiguousarray(scene.scene_id, np.int32)
        self.ij = np.ascontiguousarray(scene.ij, dtype=np.int32).reshape(-1)
        self.bmat = None if scene.bmat is None else np.ascontiguousarray(scene.bmat, np.int32)
        self.p = bdem_particles(scene.n, _p(self.pos), _p(self.quat), _p(self.vel), _p(self.qvel),
                                _p(self.radius), _p(self.pmat, _i32p), _p(self.flags, _u8p),
                                _p(self.sid, _i32p))
        self.b = bdem_bonds(scene.nb, _p(self.ij, _i32p) if scene.nb else None,
                            _p(self.bmat, _i32p))
        mats = (bdem_material * len(scene.materials))()
        for k, m in enumerate(scene.materials):
            mats[k].young, mats[k].poisson, mats[k].density = m["young"], m["poisson"], m["density"]
            mats[k].sigma_c, mats[k].tau_c = m["sigma_c"], m["tau_c"]
            mats[k].stiff_scale[:] = list(m["stiff_scale"])
            mats[k].shear_mode, mats[k].tension_only = m["shear_mode"], m["tension_only"]
        self.mats = mats


def scene_options(scene, **overrides):
    o = bdem_default_options(gravity=scene.gravity, ground_normal=scene.ground_normal,
                             ground_offset=scene.ground_offset, k_contact=scene.k_contact,
                             k_self=scene.k_self, contact_margin=scene.contact_margin,
                             mu_s=scene.mu_s, mu_r=scene.mu_r)
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def bdem_workspace_bytes(scene, opts):
    inp = _Inputs(scene)
    return _lib.bdem_workspace_bytes(C.byref(inp.p), C.byref(inp.b), C.byref(opts))


def bdem_create(scene, opts, stream=None, workspace=None):
    """Create a handle from a scene (paper_2308_10459_amd.scenes.Scene).
    workspace: a torch uint8 device tensor of at least bdem_workspace_bytes, or None."""
    inp = _Inputs(scene)
    ctx = _ctx_p()
    wptr = None if workspace is None else C.c_void_p(workspace.data_ptr())
    wbytes = 0 if workspace is None else workspace.numel()
    sptr = None if stream is None else C.c_void_p(stream.cuda_stream)
    rc = _lib.bdem_create(C.byref(inp.p), C.byref(inp.b), inp.mats, len(scene.materials),
                          C.byref(opts), sptr, wptr, wbytes, C.byref(ctx))
    _check(rc)
    return ctx


def bdem_create_in_scratch(scene, opts, stream=None):
    """Create a handle whose workspace is the library's static device array
    (no allocation; one such handle per device at a time)."""
    inp = _Inputs(scene)
    ctx = _ctx_p()
    sptr = None if stream is None else C.c_void_p(stream.cuda_stream)
    rc = _lib.bdem_create_in_scratch(C.byref(inp.p), C.byref(inp.b), inp.mats, len(scene.materials),
                                     C.byref(opts), sptr, C.byref(ctx))
    _check(rc)
    return ctx


def bdem_step(ctx, dt):
    st = bdem_step_stats()
    rc = _check(_lib.bdem_step(ctx, float(dt), C.byref(st)), ctx)
    d = st.as_dict()
    d["rc"] = rc
    return d


def bdem_step_batched(ctx, dts):
    n_scenes = bdem_sizes(ctx)[2]
    dts = _f64(dts)
    sts = (bdem_step_stats * n_scenes)()
    rc = _check(_lib.bdem_step_batched(ctx, _p(dts), sts), ctx)
    return rc, [s.as_dict() for s in sts]


def bdem_energy_grad_hess(ctx, dt, what, pos=None, quat=None):
    n, nb, _ = bdem_sizes(ctx)
    e = C.c_double()
    g = np.empty((n, 6)) if what & BDEM_EGH_G else None
    hd = np.empty((n, 6, 6)) if what & BDEM_EGH_H else None
    ho = np.empty((max(nb, 1), 6, 6)) if what & BDEM_EGH_H else None
    pos, quat = _f64(pos), _f64(quat)
    _check(_lib.bdem_energy_grad_hess(ctx, float(dt), int(what), _p(pos), _p(quat), C.byref(e),
                                      _p(g), _p(hd), _p(ho)), ctx)
    return e.value, g, hd, (None if ho is None else ho[:nb])


def bdem_precond_apply(ctx, dt, vec6, pos=None, quat=None):
    """M^-1 vec6 with the configured preconditioner at the evaluation state."""
    n = bdem_sizes(ctx)[0]
    x = _f64(np.asarray(vec6).reshape(n, 6))
    out = np.empty((n, 6))
    pe = None if pos is None else _f64(pos)
    qe = None if quat is None else _f64(quat)
    _check(_lib.bdem_precond_apply(ctx, dt, _p(pe), _p(qe), _p(x), _p(out)), ctx)
    return out


def bdem_hess_apply(ctx, dt, vec6, pos=None, quat=None):
    """H vec6 with the PCG's matrix (projected reduced Hessian) at the evaluation state."""
    n = bdem_sizes(ctx)[0]
    x = _f64(np.asarray(vec6).reshape(n, 6))
    out = np.empty((n, 6))
    pe = None if pos is None else _f64(pos)
    qe = None if quat is None else _f64(quat)
    _check(_lib.bdem_hess_apply(ctx, dt, _p(pe), _p(qe), _p(x), _p(out)), ctx)
    return out


def bdem_contact_pairs(ctx):
    """Element-repulsion candidate pairs of the last step (user indices, i < j)."""
    k = C.c_int64()
    _check(_lib.bdem_contact_pairs(ctx, 0, None, C.byref(k)), ctx)
    out = np.zeros((k.value, 2), dtype=np.int32)
    if k.value:
        _check(_lib.bdem_contact_pairs(ctx, k.value, _p(out, _i32p), C.byref(k)), ctx)
    return out


def bdem_break_bonds(ctx):
    n, nb, _ = bdem_sizes(ctx)
    k = C.c_int64()
    alive = np.empty(max(nb, 1), dtype=np.uint8)
    _check(_lib.bdem_break_bonds(ctx, C.byref(k), _p(alive, _u8p)), ctx)
    return k.value, alive[:nb]


def bdem_get_state(ctx):
    n, nb, _ = bdem_sizes(ctx)
    pos, quat, vel, qvel = np.empty((n, 3)), np.empty((n, 4)), np.empty((n, 3)), np.empty((n, 4))
    alive = np.empty(max(nb, 1), dtype=np.uint8)
    _check(_lib.bdem_get_state(ctx, _p(pos), _p(quat), _p(vel), _p(qvel), _p(alive, _u8p)), ctx)
    return dict(pos=pos, quat=quat, vel=vel, qvel=qvel, alive=alive[:nb])


def bdem_set_state(ctx, pos=None, quat=None, vel=None, qvel=None, alive=None):
    a = [_f64(x) for x in (pos, quat, vel, qvel)]
    al = None if alive is None else np.ascontiguousarray(alive, dtype=np.uint8)
    return _check(_lib.bdem_set_state(ctx, *[_p(x) for x in a], _p(al, _u8p)), ctx)


def bdem_sizes(ctx):
    n, nb, ns = C.c_int32(), C.c_int64(), C.c_int32()
    _check(_lib.bdem_sizes(ctx, C.byref(n), C.byref(nb), C.byref(ns)), ctx)
    return n.value, nb.value, ns.value


def bdem_set_profiling(ctx, enable):
    return _check(_lib.bdem_set_profiling(ctx, 1 if enable else 0), ctx)


def bdem_profile_counts(ctx):
    a, b = C.c_int32(), C.c_int32()
    _check(_lib.bdem_profile_counts(ctx, C.byref(a), C.byref(b)), ctx)
    return a.value, b.value


def bdem_autotune(ctx, dt_per_scene):
    dts = np.ascontiguousarray(np.atleast_1d(dt_per_scene), dtype=np.float64)
    t = bdem_tuning()
    _check(_lib.bdem_autotune(ctx, dts.ctypes.data_as(_dp), C.byref(t)), ctx)
    return t.as_dict()


def bdem_get_tuning(ctx):
    t = bdem_tuning()
    _check(_lib.bdem_get_tuning(ctx, C.byref(t)), ctx)
    return t.as_dict()


def bdem_set_tuning(ctx, **kw):
    t = bdem_tuning()
    _check(_lib.bdem_get_tuning(ctx, C.byref(t)), ctx)
    for k, v in kw.items():
        setattr(t, k, v)
    return _check(_lib.bdem_set_tuning(ctx, C.byref(t)), ctx)


def bdem_destroy(ctx):
    _lib.bdem_destroy(ctx)


class Simulator:
    """A handle plus its torch-owned workspace on the current device / stream."""

    def __init__(self, scene, precision=BDEM_PREC_FP64, device="cuda", stream=None, in_scratch=False,
                 **opts):
        """in_scratch: create with bdem_create_in_scratch (the library's static
        device array, no workspace tensor)."""
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the bdem library needs a GPU")
        self.scene = scene
        self.opts = scene_options(scene, precision=precision, **opts)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        if in_scratch:
            self.workspace = None
            self.ctx = bdem_create_in_scratch(scene, self.opts, self.stream)
            return
        nbytes = bdem_workspace_bytes(scene, self.opts)
        if nbytes == 0:
            raise BdemError(BDEM_E_INVALID, "invalid scene")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.ctx = bdem_create(scene, self.opts, self.stream, self.workspace)

    def step(self, dt=None):
        return bdem_step(self.ctx, self.scene.dt if dt is None else dt)

    def step_batched(self, dts=None):
        return bdem_step_batched(self.ctx, self.scene.dt_per_scene if dts is None else dts)

    def energy_grad_hess(self, dt, what, pos=None, quat=None):
        return bdem_energy_grad_hess(self.ctx, dt, what, pos, quat)

    def break_bonds(self):
        return bdem_break_bonds(self.ctx)

    def contact_pairs(self):
        return bdem_contact_pairs(self.ctx)

    def precond_apply(self, dt, vec6, pos=None, quat=None):
        return bdem_precond_apply(self.ctx, dt, vec6, pos, quat)

    def hess_apply(self, dt, vec6, pos=None, quat=None):
        return bdem_hess_apply(self.ctx, dt, vec6, pos, quat)

    def autotune(self, dts=None):
        if dts is None:
            dts = self.scene.dt_per_scene if self.scene.dt_per_scene is not None else [self.scene.dt]
        return bdem_autotune(self.ctx, dts)

    def get_tuning(self):
        return bdem_get_tuning(self.ctx)

    def set_tuning(self, **kw):
        return bdem_set_tuning(self.ctx, **kw)

    def get_state(self):
        return bdem_get_state(self.ctx)

    def set_state(self, **kw):
        return bdem_set_state(self.ctx, **kw)

    def close(self):
        if getattr(self, "ctx", None):
            bdem_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
