"""FP64 CPU oracle for the indentation solve (ctypes binding over oracle.c).

TEST INFRASTRUCTURE ONLY: the plain reference the device path is checked
against. Only the tests, the smoke check and the benchmark's CPU-baseline leg
import this package; the product path never does and must not.

Everything here marshals arguments into liboracle.so; the arithmetic lives in
oracle.c, which follows paper Sec. III-A with the readings listed there.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_SANITIZED=1 loads the build with the address and undefined-behaviour
# sanitizers (build(sanitize=True); the process needs libasan preloaded).
SANITIZED = os.environ.get("ORACLE_SANITIZED", "0") == "1"
LIB_PATH = os.path.join(HERE, "liboracle_san.so" if SANITIZED else "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")

SPHERE, CYLINDER, BOX, RING = 0, 1, 2, 3
NEOHOOKEAN, COROTATIONAL = 0, 1
OK, NOT_CONVERGED, INVERSION, NOT_SPD = 0, -6, -7, -9


def build(force: bool = True, sanitize: bool | None = None) -> str:
    """Compile oracle.c into liboracle.so (plain IEEE double: no fast-math,
    no FMA contraction), or with sanitize into liboracle_san.so, instrumented
    by the address and undefined-behaviour sanitizers (host code only)."""
    if sanitize is None:
        sanitize = SANITIZED
    path = os.path.join(HERE, "liboracle_san.so" if sanitize else "liboracle.so")
    if force or not os.path.exists(path):
        opt = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all"] if sanitize else ["-O3"]
        cmd = ["gcc", *opt, "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
               "-Wall", "-fPIC", "-shared", "-o", path + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(path + ".tmp", path)
    return path


class Indenter(C.Structure):
    _fields_ = [("kind", C.c_int), ("shape", C.c_double * 4), ("R", C.c_double * 9),
                ("c", C.c_double * 3), ("k", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("n", C.c_int), ("m", C.c_int), ("X", C.POINTER(C.c_double)), ("T", C.POINTER(C.c_int)),
                ("fixed", C.POINTER(C.c_ubyte)), ("eligible", C.POINTER(C.c_ubyte)),
                ("B", C.POINTER(C.c_double)), ("V", C.POINTER(C.c_double)),
                ("mu", C.c_double), ("lam", C.c_double), ("ind", Indenter), ("dt", C.c_double),
                ("mass", C.POINTER(C.c_double)), ("utilde", C.POINTER(C.c_double)), ("model", C.c_int),
                ("mu_f", C.c_double), ("eps_f", C.c_double), ("u_lag", C.POINTER(C.c_double)),
                ("c_lag", C.c_double * 3)]


class Params(C.Structure):
    _fields_ = [("newton_rtol", C.c_double), ("newton_atol", C.c_double), ("max_newton", C.c_int),
                ("cg_rtol", C.c_double), ("cg_eta_max", C.c_double), ("max_cg", C.c_int),
                ("precond", C.c_int), ("c1", C.c_double), ("max_halvings", C.c_int), ("dense", C.c_int),
                ("contact_hessian", C.c_int)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int), ("newton_iters", C.c_int), ("cg_iters", C.c_int), ("ls_trials", C.c_int),
                ("grad_passes", C.c_int), ("energy_passes", C.c_int), ("hv_products", C.c_int),
                ("g0_norm", C.c_double), ("g_norm", C.c_double), ("energy", C.c_double), ("min_J", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        L = C.CDLL(LIB_PATH)
        dp, ip, up = C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_ubyte)
        L.orc_lame.argtypes = [C.c_double, C.c_double, dp, dp]
        L.orc_psi.argtypes = [dp, C.c_double, C.c_double]
        L.orc_psi.restype = C.c_double
        L.orc_pk1.argtypes = [dp, C.c_double, C.c_double, dp]
        L.orc_dpk1.argtypes = [dp, dp, C.c_double, C.c_double, dp]
        L.orc_sdf.argtypes = [C.POINTER(Indenter), dp, dp]
        L.orc_sdf.restype = C.c_double
        L.orc_precompute.argtypes = [C.c_int, dp, C.c_int, ip, dp, dp]
        L.orc_surface_nodes.argtypes = [C.c_int, C.c_int, ip, up]
        L.orc_lumped_mass.argtypes = [C.c_int, C.c_int, ip, dp, C.c_double, dp]
        L.orc_lumped_mass.restype = None
        L.orc_polar.argtypes = [dp, dp, dp]
        L.orc_friction_f0.argtypes = [C.c_double, C.c_double, dp, dp, dp]
        L.orc_friction_f0.restype = None
        L.orc_psi_cr.argtypes = [dp, C.c_double, C.c_double]
        L.orc_psi_cr.restype = C.c_double
        L.orc_pk1_cr.argtypes = [dp, C.c_double, C.c_double, dp]
        L.orc_dpk1_cr.argtypes = [dp, dp, C.c_double, C.c_double, dp]
        L.orc_cauchy.argtypes = [dp, C.c_double, C.c_double, dp, dp]
        L.orc_cauchy.restype = None
        L.orc_tet_stress.argtypes = [C.POINTER(Problem), dp, dp, dp]
        L.orc_tet_stress.restype = None
        L.orc_displacement_stats.argtypes = [C.c_int, dp, dp, dp]
        L.orc_displacement_stats.restype = None
        L.orc_deformation_gradient.argtypes = [C.POINTER(Problem), dp, C.c_int, dp]
        L.orc_energy.argtypes = [C.POINTER(Problem), dp, dp]
        L.orc_energy.restype = C.c_double
        L.orc_gradient.argtypes = [C.POINTER(Problem), dp, dp]
        L.orc_hessian_dense.argtypes = [C.POINTER(Problem), dp, dp, C.c_int]
        L.orc_hessvec.argtypes = [C.POINTER(Problem), dp, dp, dp, C.c_int]
        L.orc_linear_solve.argtypes = [C.POINTER(Problem), dp, dp, dp, C.POINTER(Params), C.c_double]
        L.orc_step.argtypes = [C.POINTER(Problem), C.POINTER(Params), dp, C.POINTER(Info)]
        L.orc_contact_patch.argtypes = [C.POINTER(Problem), dp, ip, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def lame(E, nu):
    mu, lam = C.c_double(), C.c_double()
    lib().orc_lame(E, nu, C.byref(mu), C.byref(lam))
    return mu.value, lam.value


def psi(F, mu, lam):
    return lib().orc_psi(_dp(_f64(F, (3, 3))), mu, lam)


def pk1(F, mu, lam):
    P = np.zeros((3, 3))
    lib().orc_pk1(_dp(_f64(F, (3, 3))), mu, lam, _dp(P))
    return P


def dpk1(F, dF, mu, lam):
    dP = np.zeros((3, 3))
    lib().orc_dpk1(_dp(_f64(F, (3, 3))), _dp(_f64(dF, (3, 3))), mu, lam, _dp(dP))
    return dP


def make_indenter(kind, shape, R=None, c=(0.0, 0.0, 0.0), k=1.0e4) -> Indenter:
    ind = Indenter()
    ind.kind = int(kind)
    sh = list(np.asarray(shape, dtype=np.float64).ravel()) + [0.0] * 4
    for i in range(4):
        ind.shape[i] = sh[i]
    Rm = np.eye(3) if R is None else np.asarray(R, dtype=np.float64)
    for i, v in enumerate(Rm.ravel()):
        ind.R[i] = v
    for i in range(3):
        ind.c[i] = float(c[i])
    ind.k = float(k)
    return ind


def sdf(ind: Indenter, x):
    g = np.zeros(3)
    phi = lib().orc_sdf(C.byref(ind), _dp(_f64(x, (3,))), _dp(g))
    return phi, g


def precompute(X, tets):
    X = _f64(X)
    T = np.ascontiguousarray(tets, dtype=np.int32)
    m = T.shape[0]
    B = np.zeros((m, 3, 3))
    V = np.zeros(m)
    rc = lib().orc_precompute(X.shape[0], _dp(X), m, T.ctypes.data_as(C.POINTER(C.c_int)), _dp(B), _dp(V))
    return rc, B, V


def surface_nodes(n, tets):
    T = np.ascontiguousarray(tets, dtype=np.int32)
    s = np.zeros(n, dtype=np.uint8)
    nb = lib().orc_surface_nodes(n, T.shape[0], T.ctypes.data_as(C.POINTER(C.c_int)),
                                 s.ctypes.data_as(C.POINTER(C.c_ubyte)))
    return s, nb


def polar(F):
    R, S = np.zeros((3, 3)), np.zeros((3, 3))
    rc = lib().orc_polar(_dp(_f64(F, (3, 3))), _dp(R), _dp(S))
    return rc, R, S


def psi_cr(F, mu, lam):
    return lib().orc_psi_cr(_dp(_f64(F, (3, 3))), mu, lam)


def pk1_cr(F, mu, lam):
    P = np.zeros((3, 3))
    lib().orc_pk1_cr(_dp(_f64(F, (3, 3))), mu, lam, _dp(P))
    return P


def dpk1_cr(F, dF, mu, lam):
    dP = np.zeros((3, 3))
    lib().orc_dpk1_cr(_dp(_f64(F, (3, 3))), _dp(_f64(dF, (3, 3))), mu, lam, _dp(dP))
    return dP


def cauchy(F, mu, lam):
    """(sigma as xx yy zz xy xz yz, von Mises) of one deformation gradient."""
    s = np.zeros(6)
    vm = C.c_double()
    lib().orc_cauchy(_dp(_f64(F, (3, 3))), mu, lam, _dp(s), C.byref(vm))
    return s, vm.value


def displacement_stats(u):
    u = _f64(u).reshape(-1, 3)
    mx, mean = C.c_double(), C.c_double()
    lib().orc_displacement_stats(int(u.shape[0]), _dp(u), C.byref(mx), C.byref(mean))
    return mx.value, mean.value


def lumped_mass(n, tets, V, rho):
    m = np.zeros(n)
    T = np.ascontiguousarray(tets, dtype=np.int32)
    lib().orc_lumped_mass(int(n), int(T.shape[0]), T.ctypes.data_as(C.POINTER(C.c_int)), _dp(_f64(V)),
                          float(rho), _dp(m))
    return m


def friction_f0(y, eps):
    """Friction smoothing f0(y), f1(y) = f0'(y), f1'(y) at slip y."""
    f0, f1, df1 = C.c_double(), C.c_double(), C.c_double()
    lib().orc_friction_f0(float(y), float(eps), C.byref(f0), C.byref(f1), C.byref(df1))
    return f0.value, f1.value, df1.value


def default_params(**kw) -> Params:
    """Oracle solve settings: Newton to 1e-8 relative residual, CG forcing
    between 1e-8 and 0.1, block Jacobi, Armijo c1 = 1e-4, 40 halvings."""
    p = Params(newton_rtol=1e-8, newton_atol=1e-14, max_newton=50, cg_rtol=1e-8, cg_eta_max=0.1,
               max_cg=100000, precond=1, c1=1e-4, max_halvings=40, dense=0, contact_hessian=1)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Solver:
    """One mesh + material + indenter; keeps the arrays the C struct points to."""

    def __init__(self, X, tets, fixed, E=0.3e6, nu=0.45):
        self.X = _f64(X)
        self.T = np.ascontiguousarray(tets, dtype=np.int32)
        self.fixed = np.ascontiguousarray(fixed, dtype=np.uint8)
        self.n, self.m = self.X.shape[0], self.T.shape[0]
        rc, self.B, self.V = precompute(self.X, self.T)
        if rc != 0:
            raise ValueError(f"degenerate tet {-rc - 1}")
        surf, self.n_boundary_faces = surface_nodes(self.n, self.T)
        self.surface = surf
        self.eligible = np.ascontiguousarray(((surf == 1) & (self.fixed == 0)).astype(np.uint8))
        self.p = Problem()
        self.p.n, self.p.m = self.n, self.m
        self.p.X = _dp(self.X)
        self.p.T = self.T.ctypes.data_as(C.POINTER(C.c_int))
        self.p.fixed = self.fixed.ctypes.data_as(C.POINTER(C.c_ubyte))
        self.p.eligible = self.eligible.ctypes.data_as(C.POINTER(C.c_ubyte))
        self.p.B = _dp(self.B)
        self.p.V = _dp(self.V)
        self.set_material(E, nu)
        self.p.ind = make_indenter(SPHERE, [0.0], c=(1e9, 1e9, 1e9), k=0.0)
        self.dt = 0.0
        self.mass = None
        self.utilde = np.zeros((self.n, 3))
        self.mu_f, self.eps_f, self.u_lag = 0.0, 1e-5, None

    def set_model(self, model):
        """Constitutive law: NEOHOOKEAN (default) or COROTATIONAL."""
        self.p.model = int(model)

    def set_friction(self, mu_f, eps=1e-5):
        """Lagged, smoothed Coulomb friction (mu_f = 0: frictionless)."""
        self.mu_f, self.eps_f = float(mu_f), float(eps)
        self.p.mu_f, self.p.eps_f = self.mu_f, self.eps_f

    def set_friction_lag(self, u_lag, c_lag):
        """The lag state friction takes its normal forces and normals from:
        displacement u_lag with the indenter centred at c_lag (same shape,
        orientation and stiffness as the current indenter). None clears it."""
        if u_lag is None:
            self.u_lag = None
            self.p.u_lag = None
            return
        self.u_lag = self._u(u_lag).copy()
        self.p.u_lag = _dp(self.u_lag)
        for d in range(3):
            self.p.c_lag[d] = float(c_lag[d])

    def set_dynamics(self, dt, rho):
        """Backward-Euler time stepping with lumped masses (dt = 0: quasi-static)."""
        self.dt = float(dt)
        self.mass = lumped_mass(self.n, self.T, self.V, rho)
        self.p.dt = self.dt
        self.p.mass = _dp(self.mass) if dt > 0 else None
        self.p.utilde = _dp(self.utilde) if dt > 0 else None

    def dyn_step(self, u, v, params=None):
        """One backward-Euler step from (u, v) (not modified) at the current
        indenter pose: ut = u + dt v, Newton on the incremental potential from
        u, then v_new = (u_new - u) / dt. Returns (u_new, v_new, info)."""
        if not self.dt > 0:
            raise ValueError("set_dynamics(dt > 0, rho) first")
        u = self._u(u)
        self.utilde[...] = u + self.dt * self._u(v)
        un, info = self.step(u, params)
        return un, (un - u) / self.dt, info

    def solve_dynamic(self, ind, dt, rho, params=None, steps=None, u0=None, v0=None):
        """Time steps of a workload Indentation with the indenter at
        ind.center(k) at step k; returns the list of (u, v, info)."""
        self.set_dynamics(dt, rho)
        u = np.zeros((self.n, 3)) if u0 is None else self._u(u0).copy()
        v = np.zeros((self.n, 3)) if v0 is None else self._u(v0).copy()
        out = []
        S = ind.steps if steps is None else steps
        for k in range(1, S + 1):
            self.set_indenter(ind.kind, ind.shape, ind.R, ind.center(k), ind.k_penalty)
            if self.mu_f > 0.0:
                self.set_friction_lag(u, ind.center(k - 1))
            u, v, info = self.dyn_step(u, v, params)
            out.append((u, v, info))
        return out

    def set_material(self, E, nu):
        self.mu, self.lam = lame(E, nu)
        self.p.mu, self.p.lam = self.mu, self.lam

    def set_indenter(self, kind, shape, R, c, k=1.0e4):
        self.p.ind = make_indenter(kind, shape, R, c, k)

    def _u(self, u):
        return _f64(u, (self.n, 3))

    def energy(self, u):
        mj = C.c_double()
        e = lib().orc_energy(C.byref(self.p), _dp(self._u(u)), C.byref(mj))
        return e, mj.value

    def gradient(self, u):
        g = np.zeros((self.n, 3))
        lib().orc_gradient(C.byref(self.p), _dp(self._u(u)), _dp(g))
        return g

    def deformation_gradient(self, u, e):
        F = np.zeros((3, 3))
        lib().orc_deformation_gradient(C.byref(self.p), _dp(self._u(u)), int(e), _dp(F))
        return F

    def hessian_dense(self, u, contact_full=1):
        N = 3 * self.n
        H = np.zeros((N, N))
        lib().orc_hessian_dense(C.byref(self.p), _dp(self._u(u)), _dp(H), int(contact_full))
        return H

    def hessvec(self, u, v, contact_full=1):
        q = np.zeros((self.n, 3))
        lib().orc_hessvec(C.byref(self.p), _dp(self._u(u)), _dp(self._u(v)), _dp(q), int(contact_full))
        return q

    def linear_solve(self, u, b, params=None, rtol=1e-12):
        prm = params or default_params()
        x = np.zeros((self.n, 3))
        rc = lib().orc_linear_solve(C.byref(self.p), _dp(self._u(u)), _dp(self._u(b)), _dp(x), C.byref(prm), rtol)
        return rc, x

    def step(self, u, params=None):
        """One load step from u (not modified); returns (u_new, info dict)."""
        prm = params or default_params()
        un = self._u(u).copy()
        info = Info()
        lib().orc_step(C.byref(self.p), C.byref(prm), _dp(un), C.byref(info))
        return un, info.as_dict()

    def tet_stress(self, u):
        """Per-tet Cauchy stress (m x 6: xx yy zz xy xz yz) and von Mises (m)."""
        sig = np.zeros((self.m, 6))
        vm = np.zeros(self.m)
        lib().orc_tet_stress(C.byref(self.p), _dp(self._u(u)), _dp(sig), _dp(vm))
        return sig, vm

    def contact_patch(self, u):
        uu = self._u(u)
        cnt = lib().orc_contact_patch(C.byref(self.p), _dp(uu), None, None, None, None)
        ids = np.zeros(max(cnt, 1), dtype=np.int32)
        f = np.zeros((max(cnt, 1), 3))
        phi = np.zeros(max(cnt, 1))
        Ft = np.zeros(3)
        lib().orc_contact_patch(C.byref(self.p), _dp(uu), ids.ctypes.data_as(C.POINTER(C.c_int)), _dp(f), _dp(phi),
                                _dp(Ft))
        return ids[:cnt], f[:cnt], phi[:cnt], Ft

    def solve_indentation(self, ind, E=None, nu=None, params=None, steps=None, u0=None, callback=None):
        """Runs the load steps of a workload Indentation; returns the list of
        (u, info) per step. `steps` limits how many load steps are taken."""
        if E is not None:
            self.set_material(E, nu)
        u = np.zeros((self.n, 3)) if u0 is None else self._u(u0).copy()
        out = []
        S = ind.steps if steps is None else steps
        for k in range(1, S + 1):
            self.set_indenter(ind.kind, ind.shape, ind.R, ind.center(k), ind.k_penalty)
            if self.mu_f > 0.0:
                # friction lagged from the previous load step's result
                self.set_friction_lag(u, ind.center(k - 1))
            u, info = self.step(u, params)
            out.append((u, info))
            if callback:
                callback(k, u, info)
        return out


@dataclass
class StepResult:
    u: np.ndarray
    info: dict
