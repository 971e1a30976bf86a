"""ctypes wrapper of the plain-C FP64 oracle (``iblbm_oracle.c``).

Test infrastructure only: see the package docstring.  The C source is built
with ``gcc -O2 -ffp-contract=off`` (no fast-math, no FMA contraction) so its
rounding is the plain IEEE double rounding of each written operation.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "iblbm_oracle.c")
_LIB = os.path.join(_HERE, "libiblbm_oracle.so")

BGK, TRT, CMMRT = 0, 1, 2
PERIODIC, BOUNCE_BACK, VEL_PARABOLIC, VEL_UNIFORM, ZERO_GRADIENT, ZOU_HE = 0, 1, 2, 3, 4, 5
DF, MDF, DFC = 0, 1, 2
HAT, PESKIN4 = 0, 1
FIXED, PRESCRIBED_SIN, FREE = 0, 1, 2
IM_NONE, IM_FENG = 0, 1
VERLET, EULER_A1 = 0, 1
UD_RIGID, UD_TAYLOR_GREEN = 0, 1


def build_oracle(force: bool = True) -> str:
    """Compile the oracle shared library next to its source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-D_DEFAULT_SOURCE",
               "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("collision", C.c_int32), ("pad0", C.c_int32),
                ("tau", C.c_double), ("trt_magic", C.c_double), ("cm_s_q", C.c_double),
                ("cm_s_eps", C.c_double), ("rho0", C.c_double), ("bc", C.c_int32 * 4),
                ("u_bc", C.c_double), ("gravity", C.c_double * 2), ("fluid_force", C.c_double * 2)]


class _Body(C.Structure):
    _fields_ = [("xc", C.c_double), ("yc", C.c_double), ("diameter", C.c_double),
                ("n_markers", C.c_int32), ("scheme", C.c_int32), ("kernel", C.c_int32),
                ("mdf_iters", C.c_int32), ("mdf_omega", C.c_double), ("motion", C.c_int32),
                ("internal_mass", C.c_int32), ("amp", C.c_double * 2), ("freq", C.c_double),
                ("phase", C.c_double), ("density_ratio", C.c_double),
                ("mdf_nmin", C.c_int32), ("pad1", C.c_int32), ("mdf_tol", C.c_double),
                ("integrator", C.c_int32), ("mdf_coupled", C.c_int32),
                ("udes", C.c_int32), ("pad2", C.c_int32), ("tg_u0", C.c_double),
                ("tg_k", C.c_double), ("tg_nu", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_oracle(force=True)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.POINTER(_Config)]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_add_body.argtypes = [C.c_void_p, C.POINTER(_Body)]
        L.or_step.argtypes = [C.c_void_p, C.c_int64]
        L.or_steps_done.restype = C.c_int64
        L.or_steps_done.argtypes = [C.c_void_p]
        for name in ("or_get_populations", "or_set_populations"):
            getattr(L, name).argtypes = [C.c_void_p, dp]
        L.or_get_force.argtypes = [C.c_void_p, dp, dp]
        L.or_fields.argtypes = [C.c_void_p, dp, dp, dp]
        L.or_body_state.argtypes = [C.c_void_p, C.c_int, dp]
        L.or_markers.argtypes = [C.c_void_p, C.c_int, dp]
        L.or_body_omega.restype = C.c_double
        L.or_body_omega.argtypes = [C.c_void_p, C.c_int]
        L.or_mdf_residuals.restype = C.c_int
        L.or_mdf_residuals.argtypes = [C.c_void_p, C.c_int, dp]
        L.or_diagnostics.restype = C.c_int
        L.or_diagnostics.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, dp, dp]
        L.or_phi.restype = C.c_double
        L.or_phi.argtypes = [C.c_int, C.c_double]
        L.or_equilibrium.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.or_collide_node.argtypes = [C.POINTER(_Config), dp, C.c_double, C.c_double, dp]
        L.or_interp.restype = C.c_double
        L.or_interp.argtypes = [C.c_int, C.c_int, dp, C.c_double, C.c_double]
        L.or_spread.argtypes = [C.c_int, C.c_int, dp, C.c_double, C.c_double, C.c_double, C.c_double]
        L.or_dense_A.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_int, dp]
        L.or_dfc_lambda.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_int, dp]
        L.or_body_half_kick.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, dp, dp]
        L.or_body_euler.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, dp, dp]
        L.or_body_full_kick.argtypes = [C.c_double, C.c_double, C.c_double, dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_config(cfg: dict) -> _Config:
    c = _Config()
    c.nx, c.ny = int(cfg["nx"]), int(cfg["ny"])
    c.collision = int(cfg.get("collision", BGK))
    c.tau = float(cfg["tau"])
    c.trt_magic = float(cfg.get("trt_magic", 0.25))
    c.cm_s_q = float(cfg.get("cm_s_q", 1.2))
    c.cm_s_eps = float(cfg.get("cm_s_eps", 1.4))
    c.rho0 = float(cfg.get("rho0", 1.0))
    for i, b in enumerate(cfg.get("bc", (PERIODIC,) * 4)):
        c.bc[i] = int(b)
    c.u_bc = float(cfg.get("u_bc", 0.0))
    g = cfg.get("gravity", (0.0, 0.0))
    c.gravity[0], c.gravity[1] = float(g[0]), float(g[1])
    ff = cfg.get("fluid_force", (0.0, 0.0))
    c.fluid_force[0], c.fluid_force[1] = float(ff[0]), float(ff[1])
    return c


def make_body(b: dict) -> _Body:
    d = _Body()
    d.xc, d.yc, d.diameter = float(b["xc"]), float(b["yc"]), float(b["diameter"])
    d.n_markers = int(b.get("n_markers", 0))
    d.scheme = int(b.get("scheme", DF))
    d.kernel = int(b.get("kernel", HAT))
    d.mdf_iters = int(b.get("mdf_iters", 5))
    d.mdf_omega = float(b.get("mdf_omega", 0.0))
    d.motion = int(b.get("motion", FIXED))
    d.internal_mass = int(b.get("internal_mass", IM_NONE))
    amp = b.get("amp", (0.0, 0.0))
    d.amp[0], d.amp[1] = float(amp[0]), float(amp[1])
    d.freq = float(b.get("freq", 0.0))
    d.phase = float(b.get("phase", 0.0))
    d.density_ratio = float(b.get("density_ratio", 1.0))
    d.mdf_nmin = int(b.get("mdf_nmin", 1))
    d.mdf_tol = float(b.get("mdf_tol", 0.0))
    d.integrator = int(b.get("integrator", VERLET))
    d.mdf_coupled = int(b.get("mdf_coupled", 0))
    d.udes = int(b.get("udes", UD_RIGID))
    d.tg_u0 = float(b.get("tg_u0", 0.0))
    d.tg_k = float(b.get("tg_k", 0.0))
    d.tg_nu = float(b.get("tg_nu", 0.0))
    return d


class OracleSim:
    """One simulation held by the oracle; the dict keys follow ``ib_cases``."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self._c = make_config(cfg)
        self.nx, self.ny = self._c.nx, self._c.ny
        self.h = lib().or_create(C.byref(self._c))
        if not self.h:
            raise ValueError("oracle rejected the configuration")
        self.nbodies = 0
        self.nmarkers = []

    def close(self):
        if self.h:
            lib().or_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_body(self, body: dict) -> int:
        d = make_body(body)
        r = lib().or_add_body(self.h, C.byref(d))
        if r < 0:
            raise ValueError(f"oracle add_body failed ({r})")
        self.nbodies += 1
        import math
        nb = d.n_markers if d.n_markers > 0 else int(round(math.pi * d.diameter))
        self.nmarkers.append(nb)
        return r

    def step(self, n: int = 1) -> int:
        return lib().or_step(self.h, int(n))

    @property
    def steps_done(self) -> int:
        return lib().or_steps_done(self.h)

    def populations(self) -> np.ndarray:
        f = np.empty((9, self.ny, self.nx), np.float64)
        lib().or_get_populations(self.h, _dp(f))
        return f

    def set_populations(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (9, self.ny, self.nx)
        lib().or_set_populations(self.h, _dp(f))

    def force(self):
        fx = np.empty((self.ny, self.nx)); fy = np.empty((self.ny, self.nx))
        lib().or_get_force(self.h, _dp(fx), _dp(fy))
        return fx, fy

    def fields(self):
        r = np.empty((self.ny, self.nx)); ux = np.empty_like(r); uy = np.empty_like(r)
        lib().or_fields(self.h, _dp(r), _dp(ux), _dp(uy))
        return r, ux, uy

    def body_state(self, b: int = 0) -> dict:
        o = np.zeros(16)
        lib().or_body_state(self.h, b, _dp(o))
        keys = ["step", "fx", "fy", "torque", "xc", "yc", "vx", "vy", "omega", "slip_mean",
                "slip_max", "mdf_residual", "mdf_iters", "mdf_omega"]
        return {k: float(o[i]) for i, k in enumerate(keys)}

    def markers(self, b: int = 0) -> np.ndarray:
        o = np.zeros((self.nmarkers[b], 8))
        lib().or_markers(self.h, b, _dp(o))
        return o

    def mdf_omega(self, b: int = 0) -> float:
        return lib().or_body_omega(self.h, b)

    def diagnostics(self, b: int = 0, kappa: int = 2, u_ref: float = 1.0):
        """Boundary-fidelity diagnostics (summary dict, per-marker n_b x 6)."""
        sm = np.zeros(8)
        nb = self.markers(b).shape[0]
        pm = np.zeros((nb, 6))
        dpp = C.POINTER(C.c_double)
        if lib().or_diagnostics(self.h, b, int(kappa), float(u_ref), sm.ctypes.data_as(dpp),
                                pm.ctypes.data_as(dpp)) != 0:
            raise ValueError("or_diagnostics: invalid arguments")
        keys = ["slip_mean", "slip_max", "phi_leak", "u_inside_mean", "u_inside_max",
                "n_inside", "dp_mean", "force_mean"]
        return dict(zip(keys, sm.tolist())), pm

    def mdf_residuals(self, b: int = 0) -> np.ndarray:
        """MDF residual r_n of every interpolation of the last step."""
        out = np.zeros(1024)
        n = lib().or_mdf_residuals(self.h, b, out.ctypes.data_as(C.POINTER(C.c_double)))
        return out[:n].copy()


def phi(kernel: int, r: float) -> float:
    return lib().or_phi(kernel, float(r))


def equilibrium(rho, ux, uy) -> np.ndarray:
    o = np.zeros(9)
    lib().or_equilibrium(float(rho), float(ux), float(uy), _dp(o))
    return o


def collide_node(cfg: dict, f: np.ndarray, Fx=0.0, Fy=0.0) -> np.ndarray:
    c = make_config(cfg)
    fin = np.ascontiguousarray(f, np.float64)
    out = np.zeros(9)
    lib().or_collide_node(C.byref(c), _dp(fin), float(Fx), float(Fy), _dp(out))
    return out


def interp(kernel, field: np.ndarray, X, Y) -> float:
    f = np.ascontiguousarray(field, np.float64)
    return lib().or_interp(kernel, f.shape[1], _dp(f), float(X), float(Y))


def spread(kernel, field: np.ndarray, F, X, Y, ds):
    assert field.dtype == np.float64 and field.flags.c_contiguous
    lib().or_spread(kernel, field.shape[1], _dp(field), float(F), float(X), float(Y), float(ds))


def dense_A(kernel, xc, yc, diameter, nb) -> np.ndarray:
    A = np.zeros((nb, nb))
    lib().or_dense_A(kernel, xc, yc, diameter, nb, _dp(A))
    return A


def dfc_lambda(kernel, xc, yc, diameter, nb) -> np.ndarray:
    lam = np.zeros(nb)
    lib().or_dfc_lambda(kernel, xc, yc, diameter, nb, _dp(lam))
    return lam


def body_half_kick(ms, mf, Is, internal_mass, g, st: np.ndarray):
    gv = np.ascontiguousarray(g, np.float64)
    lib().or_body_half_kick(ms, mf, Is, internal_mass, _dp(gv), _dp(st))


def body_full_kick(ms, mf, Is, g, st: np.ndarray):
    gv = np.ascontiguousarray(g, np.float64)
    lib().or_body_full_kick(ms, mf, Is, _dp(gv), _dp(st))


def body_euler(ms, mf, Is, internal_mass, g, st: np.ndarray):
    gv = np.ascontiguousarray(g, np.float64)
    lib().or_body_euler(ms, mf, Is, internal_mass, _dp(gv), _dp(st))
