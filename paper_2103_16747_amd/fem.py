"""Python binding of libfem (include/fem.h): argument marshalling only.

Every function with an ``fem_`` name calls the C entry point of the same name;
all arithmetic of the solve runs in the HIP kernels behind it. If libfem.so has
not been built this module raises on import of the library: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfem.so")

FEM_OK = 0
FEM_MODEL_NEOHOOKEAN, FEM_MODEL_COROTATIONAL = 0, 1
FEM_W_FLOOR = 1
FEM_E_INVALID, FEM_E_DEGENERATE, FEM_E_OOM, FEM_E_DEVICE = -1, -2, -3, -4
FEM_E_STATE, FEM_E_NOT_CONVERGED, FEM_E_INVERSION, FEM_E_BUFFER = -5, -6, -7, -8
FEM_PREC_FP64, FEM_PREC_FP32 = 0, 1
FEM_SPHERE, FEM_CYLINDER, FEM_BOX, FEM_RING = 0, 1, 2, 3
PRECISIONS = {"fp64": FEM_PREC_FP64, "fp32": FEM_PREC_FP32}

# Entry points declared in include/fem.h.
EXPORTS = ("fem_create_mesh", "fem_destroy_mesh", "fem_set_material", "fem_set_indenter", "fem_default_params",
           "fem_step", "fem_get_displacements", "fem_set_displacements", "fem_get_contact_patch",
           "fem_get_mesh_info", "fem_get_tet_stress", "fem_get_displacement_stats", "fem_set_model", "fem_set_friction", "fem_set_dynamics", "fem_get_velocities", "fem_set_velocities", "fem_eval_gradient", "fem_eval_hessvec", "fem_set_kernel_timing",
           "fem_get_kernel_timing", "fem_batch_create", "fem_batch_destroy", "fem_batch_add_mesh",
           "fem_batch_mesh_info", "fem_batch_add_job", "fem_batch_restart_job", "fem_batch_remove_job", "fem_batch_run", "fem_batch_job_info",
           "fem_batch_job_step_status",
           "fem_batch_get_displacements", "fem_batch_get_velocities", "fem_batch_get_tet_stress",
           "fem_batch_get_displacement_stats", "fem_batch_get_contact_patch", "fem_batch_get_contact_patch_noalloc",
           "fem_batch_set_kernel_timing",
           "fem_batch_get_kernel_timing", "fem_batch_get_kernel_launches", "fem_set_graphs", "fem_batch_set_graphs", "fem_batch_set_option",
           "fem_batch_job_footprint", "fem_status_string",
           "fem_last_error")
FEM_KERNEL_TILE, FEM_KERNEL_NODE, FEM_KERNEL_FINALIZE = 0, 1, 2
FEM_OPT_ROUND_STEPS, FEM_OPT_TILE_TETS, FEM_OPT_TILE_NODES, FEM_OPT_GROUPS, FEM_OPT_DETERMINISTIC = 0, 1, 2, 3, 4


class FemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class fem_config(C.Structure):
    _fields_ = [("precision", C.c_int32), ("device", C.c_int32), ("stream", C.c_void_p)]


class fem_solve_params(C.Structure):
    _fields_ = [("newton_rtol", C.c_double), ("newton_atol", C.c_double), ("max_newton", C.c_int32),
                ("cg_rtol", C.c_double), ("cg_eta_max", C.c_double), ("max_cg", C.c_int32),
                ("precond", C.c_int32), ("contact_hessian", C.c_int32), ("c1", C.c_double),
                ("max_halvings", C.c_int32), ("newton_floor_rtol", C.c_double), ("cg_eta_power", C.c_double)]


class fem_step_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("newton_iters", C.c_int32), ("cg_iters", C.c_int32),
                ("ls_trials", C.c_int32), ("grad_passes", C.c_int32), ("hv_products", C.c_int32),
                ("g0_norm", C.c_double), ("g_norm", C.c_double), ("energy", C.c_double), ("min_J", C.c_double),
                ("tet_updates", C.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class fem_indentation(C.Structure):
    _fields_ = [("kind", C.c_int32), ("shape", C.c_double * 4), ("R", C.c_double * 9), ("c0", C.c_double * 3),
                ("direction", C.c_double * 3), ("depth", C.c_double), ("steps", C.c_int32), ("k_penalty", C.c_double),
                ("dt", C.c_double), ("density", C.c_double), ("model", C.c_int32),
                ("friction", C.c_double), ("friction_eps", C.c_double)]


class fem_job_info(C.Structure):
    _fields_ = [("done", C.c_int32), ("status", C.c_int32), ("step", C.c_int32), ("steps_ok", C.c_int32),
                ("steps_failed", C.c_int32), ("steps_floor", C.c_int32), ("newton_iters", C.c_int64), ("cg_iters", C.c_int64),
                ("hv_products", C.c_int64), ("grad_passes", C.c_int64), ("ls_trials", C.c_int64),
                ("tet_updates", C.c_int64), ("energy", C.c_double), ("min_J", C.c_double), ("g_norm", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class fem_mesh_layout(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_tets", C.c_int32), ("n_tiles", C.c_int32), ("n_entries", C.c_int32),
                ("n_eligible", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Loads libfem.so; raises if it is missing (the product path has no
    fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2103_16747_amd.build.build()")
    L = C.CDLL(path)
    dp, i32p, u8p, vp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_uint8), C.c_void_p
    L.fem_create_mesh.argtypes = [dp, C.c_int32, i32p, C.c_int32, u8p, C.POINTER(fem_config), C.POINTER(vp)]
    L.fem_destroy_mesh.argtypes = [vp]
    L.fem_destroy_mesh.restype = None
    L.fem_set_material.argtypes = [vp, C.c_double, C.c_double, C.c_double]
    L.fem_set_indenter.argtypes = [vp, C.c_int32, dp, C.c_int32, dp, dp, C.c_double]
    L.fem_default_params.argtypes = [C.POINTER(fem_solve_params), C.c_int32]
    L.fem_default_params.restype = None
    L.fem_step.argtypes = [vp, C.POINTER(fem_solve_params), C.POINTER(fem_step_info)]
    L.fem_get_displacements.argtypes = [vp, dp, C.c_int64]
    L.fem_set_displacements.argtypes = [vp, dp, C.c_int64]
    L.fem_set_dynamics.argtypes = [vp, C.c_double]
    L.fem_set_model.argtypes = [vp, C.c_int32]
    L.fem_set_friction.argtypes = [vp, C.c_double, C.c_double]
    L.fem_get_tet_stress.argtypes = [vp, dp, dp, C.c_int64]
    L.fem_get_displacement_stats.argtypes = [vp, dp, dp]
    L.fem_batch_get_tet_stress.argtypes = [vp, C.c_int32, dp, dp, C.c_int64]
    L.fem_batch_get_displacement_stats.argtypes = [vp, C.c_int32, dp, dp]
    L.fem_get_velocities.argtypes = [vp, dp, C.c_int64]
    L.fem_set_velocities.argtypes = [vp, dp, C.c_int64]
    L.fem_batch_get_velocities.argtypes = [vp, C.c_int32, dp, C.c_int64]
    L.fem_get_contact_patch.argtypes = [vp, i32p, dp, dp, C.c_int32, i32p, dp]
    L.fem_get_mesh_info.argtypes = [vp, i32p, i32p, i32p, u8p, C.c_int32]
    L.fem_eval_gradient.argtypes = [vp, dp, C.c_int64, dp, dp]
    L.fem_eval_hessvec.argtypes = [vp, C.POINTER(fem_solve_params), dp, dp, C.c_int64]
    L.fem_set_kernel_timing.argtypes = [vp, C.c_int32]
    L.fem_get_kernel_timing.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    L.fem_batch_create.argtypes = [C.POINTER(fem_config), C.c_int32, C.POINTER(vp)]
    L.fem_batch_destroy.argtypes = [vp]
    L.fem_batch_destroy.restype = None
    L.fem_batch_add_mesh.argtypes = [vp, dp, C.c_int32, i32p, C.c_int32, u8p, i32p]
    L.fem_batch_mesh_info.argtypes = [vp, C.c_int32, C.POINTER(fem_mesh_layout)]
    L.fem_batch_add_job.argtypes = [vp, C.c_int32, C.c_double, C.c_double, C.POINTER(fem_indentation), i32p]
    L.fem_batch_restart_job.argtypes = [vp, C.c_int32, C.c_double, C.c_double, C.POINTER(fem_indentation)]
    L.fem_batch_remove_job.argtypes = [vp, C.c_int32]
    L.fem_batch_run.argtypes = [vp, C.POINTER(fem_solve_params), C.c_int32, i32p]
    L.fem_batch_job_info.argtypes = [vp, C.c_int32, C.POINTER(fem_job_info)]
    L.fem_batch_job_step_status.argtypes = [vp, C.c_int32, i32p, C.c_int32, i32p]
    L.fem_batch_get_displacements.argtypes = [vp, C.c_int32, dp, C.c_int64]
    L.fem_batch_get_contact_patch.argtypes = [vp, C.c_int32, i32p, dp, dp, C.c_int32, i32p, dp]
    L.fem_batch_get_contact_patch_noalloc.argtypes = [vp, C.c_int32, i32p, dp, dp, C.c_int32, i32p, dp]
    L.fem_batch_set_kernel_timing.argtypes = [vp, C.c_int32]
    L.fem_batch_get_kernel_timing.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    L.fem_batch_get_kernel_launches.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64)]
    L.fem_set_graphs.argtypes = [vp, C.c_int32]
    L.fem_batch_set_graphs.argtypes = [vp, C.c_int32]
    L.fem_batch_set_option.argtypes = [vp, C.c_int32, C.c_int32]
    L.fem_batch_job_footprint.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64)]
    L.fem_status_string.argtypes = [C.c_int]
    L.fem_status_string.restype = C.c_char_p
    L.fem_last_error.argtypes = []
    L.fem_last_error.restype = C.c_char_p
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(rc, allow=()):
    if rc < FEM_OK and rc not in allow:
        raise FemError(rc, load().fem_last_error().decode() or load().fem_status_string(rc).decode())
    return rc


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)   # a torch.cuda.Stream


# ---------------------------------------------------------------------------
# Same names as the C entry points
# ---------------------------------------------------------------------------
def fem_default_params(precision: int = FEM_PREC_FP64, **overrides) -> fem_solve_params:
    p = fem_solve_params()
    load().fem_default_params(C.byref(p), int(precision))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def fem_create_mesh(X, tets, fixed, precision: int = FEM_PREC_FP64, device: int = 0, stream=None) -> C.c_void_p:
    X = np.ascontiguousarray(X, dtype=np.float64)
    T = np.ascontiguousarray(tets, dtype=np.int32)
    F = np.ascontiguousarray(fixed, dtype=np.uint8)
    if X.ndim != 2 or X.shape[1] != 3 or T.ndim != 2 or T.shape[1] != 4 or F.shape != (X.shape[0],):
        raise ValueError("X must be n x 3, tets m x 4, fixed n")
    cfg = fem_config(int(precision), int(device), _stream_handle(stream))
    h = C.c_void_p()
    _check(load().fem_create_mesh(_dp(X), X.shape[0], T.ctypes.data_as(C.POINTER(C.c_int32)), T.shape[0],
                                  F.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(cfg), C.byref(h)))
    return h


def fem_destroy_mesh(h):
    load().fem_destroy_mesh(h)


def fem_set_material(h, E, nu, density=1100.0):
    _check(load().fem_set_material(h, float(E), float(nu), float(density)))


def fem_set_indenter(h, kind, shape, R, c, k_penalty=1.0e4):
    sh = np.ascontiguousarray(np.atleast_1d(shape), dtype=np.float64)
    Rm = np.ascontiguousarray(R, dtype=np.float64).reshape(9)
    cc = np.ascontiguousarray(c, dtype=np.float64).reshape(3)
    _check(load().fem_set_indenter(h, int(kind), _dp(sh), sh.size, _dp(Rm), _dp(cc), float(k_penalty)))


def fem_step(h, params: fem_solve_params | None = None) -> dict:
    """One load step. Returns the step info; FLOOR, NOT_CONVERGED and
    INVERSION are reported in info['status'] rather than raised."""
    info = fem_step_info()
    _check(load().fem_step(h, C.byref(params) if params is not None else None, C.byref(info)),
           allow=(FEM_E_NOT_CONVERGED, FEM_E_INVERSION))
    return info.as_dict()


def fem_get_displacements(h, n: int) -> np.ndarray:
    u = np.zeros((n, 3))
    _check(load().fem_get_displacements(h, _dp(u), u.size))
    return u


def fem_set_displacements(h, u):
    uu = np.ascontiguousarray(u, dtype=np.float64)
    _check(load().fem_set_displacements(h, _dp(uu), uu.size))


def fem_get_tet_stress(h, m: int):
    sig = np.zeros((m, 6))
    vm = np.zeros(m)
    _check(load().fem_get_tet_stress(h, _dp(sig), _dp(vm), m))
    return sig, vm


def fem_get_displacement_stats(h):
    mx, mean = C.c_double(), C.c_double()
    _check(load().fem_get_displacement_stats(h, C.byref(mx), C.byref(mean)))
    return mx.value, mean.value


def fem_batch_get_tet_stress(h, job: int, m: int):
    sig = np.zeros((m, 6))
    vm = np.zeros(m)
    _check(load().fem_batch_get_tet_stress(h, int(job), _dp(sig), _dp(vm), m))
    return sig, vm


def fem_batch_get_displacement_stats(h, job: int):
    mx, mean = C.c_double(), C.c_double()
    _check(load().fem_batch_get_displacement_stats(h, int(job), C.byref(mx), C.byref(mean)))
    return mx.value, mean.value


def fem_set_dynamics(h, dt: float):
    _check(load().fem_set_dynamics(h, float(dt)))


def fem_get_velocities(h, n: int) -> np.ndarray:
    v = np.zeros((n, 3))
    _check(load().fem_get_velocities(h, _dp(v), v.size))
    return v


def fem_set_velocities(h, v):
    vv = np.ascontiguousarray(v, dtype=np.float64)
    _check(load().fem_set_velocities(h, _dp(vv), vv.size))


def fem_get_contact_patch(h):
    cnt = C.c_int32()
    Ft = np.zeros(3)
    rc = load().fem_get_contact_patch(h, None, None, None, 0, C.byref(cnt), _dp(Ft))
    _check(rc, allow=(FEM_E_BUFFER,))
    k = max(cnt.value, 1)
    ids = np.zeros(k, dtype=np.int32)
    f = np.zeros((k, 3))
    phi = np.zeros(k)
    _check(load().fem_get_contact_patch(h, ids.ctypes.data_as(C.POINTER(C.c_int32)), _dp(f), _dp(phi), k,
                                        C.byref(cnt), _dp(Ft)))
    c = cnt.value
    return ids[:c], f[:c], phi[:c], Ft


def fem_get_mesh_info(h):
    n, m, ne = C.c_int32(), C.c_int32(), C.c_int32()
    _check(load().fem_get_mesh_info(h, C.byref(n), C.byref(m), C.byref(ne), None, 0))
    elig = np.zeros(n.value, dtype=np.uint8)
    _check(load().fem_get_mesh_info(h, None, None, None, elig.ctypes.data_as(C.POINTER(C.c_uint8)), n.value))
    return {"n": n.value, "m": m.value, "n_eligible": ne.value, "eligible": elig}


def fem_eval_gradient(h, n: int):
    g = np.zeros((n, 3))
    e, mj = C.c_double(), C.c_double()
    _check(load().fem_eval_gradient(h, _dp(g), g.size, C.byref(e), C.byref(mj)))
    return g, e.value, mj.value


def fem_eval_hessvec(h, v, params: fem_solve_params | None = None):
    vv = np.ascontiguousarray(v, dtype=np.float64)
    q = np.zeros_like(vv)
    _check(load().fem_eval_hessvec(h, C.byref(params) if params is not None else None, _dp(vv), _dp(q), q.size))
    return q


def fem_set_kernel_timing(h, every: int):
    _check(load().fem_set_kernel_timing(h, int(every)))


def fem_get_kernel_timing(h, kernel: int):
    """(sampled launches, summed milliseconds) of one timed kernel."""
    cnt, ms = C.c_int64(), C.c_double()
    _check(load().fem_get_kernel_timing(h, int(kernel), C.byref(cnt), C.byref(ms)))
    return cnt.value, ms.value


# ---------------------------------------------------------------------------
# Convenience object
# ---------------------------------------------------------------------------
class FemMesh:
    """Owns one libfem handle."""

    def __init__(self, X, tets, fixed, precision="fp64", device=0, stream=None):
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.n = int(np.asarray(X).shape[0])
        self.m = int(np.asarray(tets).shape[0])
        self.h = fem_create_mesh(X, tets, fixed, self.precision, device, stream)

    def close(self):
        if self.h:
            fem_destroy_mesh(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def default_params(self, **kw):
        return fem_default_params(self.precision, **kw)

    def set_material(self, E=0.3e6, nu=0.45, density=1100.0):
        fem_set_material(self.h, E, nu, density)

    def set_indenter(self, kind, shape, R, c, k_penalty=1.0e4):
        fem_set_indenter(self.h, kind, shape, R, c, k_penalty)

    def step(self, params=None):
        return fem_step(self.h, params)

    def displacements(self):
        return fem_get_displacements(self.h, self.n)

    def set_displacements(self, u):
        fem_set_displacements(self.h, u)

    def set_dynamics(self, dt):
        fem_set_dynamics(self.h, dt)

    def set_model(self, model):
        _check(load().fem_set_model(self.h, int(model)))

    def set_friction(self, mu_f, eps=1e-5):
        _check(load().fem_set_friction(self.h, float(mu_f), float(eps)))

    def tet_stress(self):
        return fem_get_tet_stress(self.h, self.m)

    def displacement_stats(self):
        return fem_get_displacement_stats(self.h)

    def velocities(self):
        return fem_get_velocities(self.h, self.n)

    def set_velocities(self, v):
        fem_set_velocities(self.h, v)

    def contact_patch(self):
        return fem_get_contact_patch(self.h)

    def info(self):
        return fem_get_mesh_info(self.h)

    def gradient(self):
        return fem_eval_gradient(self.h, self.n)

    def hessvec(self, v, params=None):
        return fem_eval_hessvec(self.h, v, params)

    def set_kernel_timing(self, every):
        fem_set_kernel_timing(self.h, every)

    def set_graphs(self, enable):
        _check(load().fem_set_graphs(self.h, int(enable)))

    def kernel_timing(self, kernel):
        return fem_get_kernel_timing(self.h, kernel)

    def solve_indentation(self, ind, params=None, steps=None, callback=None):
        """Runs the load steps of a workload Indentation; returns per-step info."""
        out = []
        S = ind.steps if steps is None else steps
        for k in range(1, S + 1):
            self.set_indenter(ind.kind, ind.shape, ind.R, ind.center(k), ind.k_penalty)
            info = self.step(params)
            out.append(info)
            if callback:
                callback(k, info)
        return out


# ---------------------------------------------------------------------------
# Batches
# ---------------------------------------------------------------------------
def fem_batch_create(max_jobs: int, precision: int = FEM_PREC_FP64, device: int = 0, stream=None) -> C.c_void_p:
    cfg = fem_config(int(precision), int(device), _stream_handle(stream))
    h = C.c_void_p()
    _check(load().fem_batch_create(C.byref(cfg), int(max_jobs), C.byref(h)))
    return h


def fem_batch_destroy(h):
    load().fem_batch_destroy(h)


def fem_batch_add_mesh(h, X, tets, fixed) -> int:
    X = np.ascontiguousarray(X, dtype=np.float64)
    T = np.ascontiguousarray(tets, dtype=np.int32)
    F = np.ascontiguousarray(fixed, dtype=np.uint8)
    mid = C.c_int32()
    _check(load().fem_batch_add_mesh(h, _dp(X), X.shape[0], T.ctypes.data_as(C.POINTER(C.c_int32)), T.shape[0],
                                     F.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(mid)))
    return mid.value


def fem_batch_mesh_info(h, mesh_id: int) -> dict:
    info = fem_mesh_layout()
    _check(load().fem_batch_mesh_info(h, int(mesh_id), C.byref(info)))
    return {name: getattr(info, name) for name, _ in info._fields_}


def make_indentation(ind) -> fem_indentation:
    """fem_indentation from a workload Indentation (or anything with the same
    attributes)."""
    j = fem_indentation()
    j.kind = int(ind.kind)
    sh = list(np.asarray(ind.shape, dtype=np.float64).ravel()) + [0.0] * 4
    for i in range(4):
        j.shape[i] = sh[i]
    for i, v in enumerate(np.asarray(ind.R, dtype=np.float64).ravel()):
        j.R[i] = v
    for i in range(3):
        j.c0[i] = float(ind.c0[i])
        j.direction[i] = float(ind.direction[i])
    j.depth = float(ind.depth)
    j.steps = int(ind.steps)
    j.k_penalty = float(ind.k_penalty)
    j.dt = float(getattr(ind, "dt", 0.0))
    j.density = float(getattr(ind, "density", 1100.0))
    j.model = int(getattr(ind, "model", FEM_MODEL_NEOHOOKEAN))
    j.friction = float(getattr(ind, "friction", 0.0))
    j.friction_eps = float(getattr(ind, "friction_eps", 1e-5))
    return j


def fem_batch_add_job(h, mesh_id: int, E: float, nu: float, ind) -> int:
    job = ind if isinstance(ind, fem_indentation) else make_indentation(ind)
    jid = C.c_int32()
    _check(load().fem_batch_add_job(h, int(mesh_id), float(E), float(nu), C.byref(job), C.byref(jid)))
    return jid.value


def fem_batch_restart_job(h, job: int, E: float, nu: float, ind):
    j = ind if isinstance(ind, fem_indentation) else make_indentation(ind)
    _check(load().fem_batch_restart_job(h, int(job), float(E), float(nu), C.byref(j)))


def fem_batch_remove_job(h, job: int):
    _check(load().fem_batch_remove_job(h, int(job)))


def fem_batch_run(h, params: fem_solve_params | None = None, max_rounds: int = 0) -> int:
    running = C.c_int32()
    _check(load().fem_batch_run(h, C.byref(params) if params is not None else None, int(max_rounds),
                                C.byref(running)))
    return running.value


def fem_batch_job_info(h, job: int) -> dict:
    info = fem_job_info()
    _check(load().fem_batch_job_info(h, int(job), C.byref(info)))
    return info.as_dict()


def fem_batch_job_step_status(h, job: int) -> np.ndarray:
    """Status of each load step the job has taken (FEM_OK, FEM_W_FLOOR,
    FEM_E_NOT_CONVERGED, FEM_E_INVERSION), in step order."""
    cnt = C.c_int32()
    _check(load().fem_batch_job_step_status(h, int(job), None, 0, C.byref(cnt)))
    st = np.zeros(max(cnt.value, 1), dtype=np.int32)
    _check(load().fem_batch_job_step_status(h, int(job), st.ctypes.data_as(C.POINTER(C.c_int32)), st.size,
                                            C.byref(cnt)))
    return st[:cnt.value]


def fem_batch_get_displacements(h, job: int, n: int) -> np.ndarray:
    u = np.zeros((n, 3))
    _check(load().fem_batch_get_displacements(h, int(job), _dp(u), u.size))
    return u


def fem_batch_get_velocities(h, job: int, n: int) -> np.ndarray:
    v = np.zeros((n, 3))
    _check(load().fem_batch_get_velocities(h, int(job), _dp(v), v.size))
    return v


def fem_batch_get_contact_patch(h, job: int):
    cnt = C.c_int32()
    Ft = np.zeros(3)
    _check(load().fem_batch_get_contact_patch(h, int(job), None, None, None, 0, C.byref(cnt), _dp(Ft)),
           allow=(FEM_E_BUFFER,))
    k = max(cnt.value, 1)
    ids = np.zeros(k, dtype=np.int32)
    f = np.zeros((k, 3))
    phi = np.zeros(k)
    _check(load().fem_batch_get_contact_patch(h, int(job), ids.ctypes.data_as(C.POINTER(C.c_int32)), _dp(f),
                                              _dp(phi), k, C.byref(cnt), _dp(Ft)))
    c = cnt.value
    return ids[:c], f[:c], phi[:c], Ft


def fem_batch_get_contact_patch_noalloc(h, job: int, ids, f, phi, F_total):
    """Allocation-free contact patch into caller arrays (ids int32, f n x 3,
    phi, F_total 3; f and phi need ids; with ids None only the count and the
    resultant are read); returns the contact count."""
    cnt = C.c_int32()
    cap = 0 if ids is None else int(ids.shape[0])
    i32 = None if ids is None else ids.ctypes.data_as(C.POINTER(C.c_int32))
    _check(load().fem_batch_get_contact_patch_noalloc(h, int(job), i32, None if f is None else _dp(f),
                                                      None if phi is None else _dp(phi), cap, C.byref(cnt),
                                                      None if F_total is None else _dp(F_total)),
           allow=(FEM_E_BUFFER,) if ids is None else ())
    return cnt.value


def fem_batch_set_kernel_timing(h, every: int):
    _check(load().fem_batch_set_kernel_timing(h, int(every)))


def fem_batch_get_kernel_timing(h, kernel: int):
    cnt, ms = C.c_int64(), C.c_double()
    _check(load().fem_batch_get_kernel_timing(h, int(kernel), C.byref(cnt), C.byref(ms)))
    return cnt.value, ms.value


def fem_batch_get_kernel_launches(h, kernel: int):
    n = C.c_int64()
    _check(load().fem_batch_get_kernel_launches(h, int(kernel), C.byref(n)))
    return n.value


class FemBatch:
    """Owns one libfem batch handle: meshes plus concurrently solved jobs."""

    def __init__(self, max_jobs, precision="fp32", device=0, stream=None):
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.h = fem_batch_create(max_jobs, self.precision, device, stream)
        self.mesh_nodes = {}
        self.mesh_tets = {}
        self.job_mesh = {}

    def close(self):
        if self.h:
            fem_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def default_params(self, **kw):
        return fem_default_params(self.precision, **kw)

    def add_mesh(self, X, tets, fixed):
        mid = fem_batch_add_mesh(self.h, X, tets, fixed)
        self.mesh_nodes[mid] = int(np.asarray(X).shape[0])
        self.mesh_tets[mid] = int(np.asarray(tets).shape[0])
        return mid

    def mesh_info(self, mesh_id):
        return fem_batch_mesh_info(self.h, mesh_id)

    def add_job(self, mesh_id, ind, E=0.3e6, nu=0.45):
        jid = fem_batch_add_job(self.h, mesh_id, E, nu, ind)
        self.job_mesh[jid] = mesh_id
        return jid

    def restart_job(self, job, ind, E=0.3e6, nu=0.45):
        fem_batch_restart_job(self.h, job, E, nu, ind)

    def remove_job(self, job):
        fem_batch_remove_job(self.h, job)
        self.job_mesh.pop(job, None)

    def run(self, params=None, max_rounds=0):
        return fem_batch_run(self.h, params, max_rounds)

    def job_info(self, job):
        return fem_batch_job_info(self.h, job)

    def step_status(self, job):
        return fem_batch_job_step_status(self.h, job)

    def displacements(self, job):
        return fem_batch_get_displacements(self.h, job, self.mesh_nodes[self.job_mesh[job]])

    def velocities(self, job):
        return fem_batch_get_velocities(self.h, job, self.mesh_nodes[self.job_mesh[job]])

    def tet_stress(self, job):
        return fem_batch_get_tet_stress(self.h, job, self.mesh_tets[self.job_mesh[job]])

    def displacement_stats(self, job):
        return fem_batch_get_displacement_stats(self.h, job)

    def contact_patch(self, job):
        return fem_batch_get_contact_patch(self.h, job)

    def contact_patch_noalloc(self, job, ids, f, phi, F_total):
        return fem_batch_get_contact_patch_noalloc(self.h, job, ids, f, phi, F_total)

    def set_kernel_timing(self, every):
        fem_batch_set_kernel_timing(self.h, every)

    def set_graphs(self, enable):
        _check(load().fem_batch_set_graphs(self.h, int(enable)))

    def set_option(self, option, value):
        _check(load().fem_batch_set_option(self.h, int(option), int(value)))

    def job_footprint(self, mesh_id):
        b = C.c_int64()
        _check(load().fem_batch_job_footprint(self.h, int(mesh_id), C.byref(b)))
        return b.value

    def kernel_timing(self, kernel):
        return fem_batch_get_kernel_timing(self.h, kernel)

    def kernel_launches(self, kernel):
        return fem_batch_get_kernel_launches(self.h, kernel)
