"""Python binding of the C ABI in ``include/ib_lbm.h`` (argument marshalling only).

Every step of the method runs in the gfx950 HIP kernels of ``libib_lbm.so``.
This module only converts Python values to the ABI's structs, passes HIP
streams and (optionally) PyTorch's caching allocator through, and raises on
error statuses.  There is no CPU fallback: if the library is missing or no
HIP device is present, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libib_lbm.so")
ABI_VERSION = 6

FP64, FP32_SHIFTED = 0, 1
BGK, TRT, CMMRT = 0, 1, 2
PERIODIC, BOUNCE_BACK, VEL_PARABOLIC, VEL_UNIFORM, ZERO_GRADIENT, ZOU_HE = 0, 1, 2, 3, 4, 5
DF, MDF, DFC = 0, 1, 2
HAT, PESKIN4 = 0, 1
FIXED, PRESCRIBED_SIN, FREE = 0, 1, 2
IM_NONE, IM_FENG = 0, 1
VERLET, EULER_A1 = 0, 1
UD_RIGID, UD_TAYLOR_GREEN = 0, 1
SPREAD_GATHER, SPREAD_ATOMIC = 0, 1
FLAG_NONFINITE, FLAG_RANGE, FLAG_OVERLAP = 1, 2, 4

PENDING = 1
MAX_BODIES = 8

STATUS = {1: "PENDING", 0: "OK", -1: "E_INVALID", -2: "E_NOMEM", -3: "E_DEVICE", -4: "E_DIVERGED",
          -5: "E_RANGE", -6: "E_STATE"}

# Exported symbols declared in include/*.h (checked by the CPU tests).
EXPORTS = [
    "ib_lbm_abi_version", "ib_lbm_create", "ib_lbm_add_body", "ib_lbm_step", "ib_lbm_forces",
    "ib_lbm_history", "ib_lbm_fields", "ib_lbm_get_populations", "ib_lbm_set_populations",
    "ib_lbm_set_equilibrium", "ib_lbm_force_field", "ib_lbm_markers", "ib_lbm_diagnostics", "ib_lbm_diagnostics_noalloc",
    "ib_lbm_steps_done",
    "ib_lbm_sync",
    "ib_lbm_destroy", "ib_lbm_last_error", "ib_lbm_footprint", "ib_lbm_set_launch",
    "ib_lbm_get_launch", "ib_lbm_set_spread", "ib_lbm_set_graph", "ib_lbm_timing_enable",
    "ib_lbm_set_overlap", "ib_lbm_get_overlap", "ib_lbm_set_fused", "ib_lbm_get_fused",
    "ib_lbm_time_collide_stream", "ib_lbm_stream_copy",
    "ib_lbm_timing_read", "ib_lbm_batch_create", "ib_lbm_batch_attach", "ib_lbm_batch_detach",
    "ib_lbm_batch_set_target", "ib_lbm_batch_step", "ib_lbm_batch_set_graph",
    "ib_lbm_batch_sync", "ib_lbm_batch_destroy", "ib_lbm_batch_last_error",
    "ib_lbm_batch_set_launch", "ib_lbm_batch_set_spread",
    "ib_lbm_server_create", "ib_lbm_server_submit", "ib_lbm_server_wait",
    "ib_lbm_server_stats_get", "ib_lbm_server_drain", "ib_lbm_server_destroy",
    "ib_lbm_server_last_error",
]


class IbLbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Allocator(C.Structure):
    _fields_ = [("ctx", C.c_void_p),
                ("alloc", C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p))]


class Config(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("precision", C.c_int32), ("collision", C.c_int32),
                ("history_capacity", C.c_int32), ("tau", C.c_double), ("trt_magic", C.c_double),
                ("cm_s_q", C.c_double), ("cm_s_eps", C.c_double), ("rho0", C.c_double),
                ("bc", C.c_int32 * 4), ("u_bc", C.c_double), ("gravity", C.c_double * 2),
                ("fluid_force", C.c_double * 2), ("stream", C.c_void_p),
                ("alloc", C.POINTER(Allocator))]


class BodyDesc(C.Structure):
    _fields_ = [("xc", C.c_double), ("yc", C.c_double), ("diameter", C.c_double),
                ("n_markers", C.c_int32), ("scheme", C.c_int32), ("kernel", C.c_int32),
                ("mdf_iters", C.c_int32), ("mdf_omega", C.c_double), ("motion", C.c_int32),
                ("internal_mass", C.c_int32), ("amp", C.c_double * 2), ("freq", C.c_double),
                ("phase", C.c_double), ("density_ratio", C.c_double),
                ("mdf_nmin", C.c_int32), ("mdf_tol", C.c_double), ("integrator", C.c_int32),
                ("mdf_coupled", C.c_int32), ("udes", C.c_int32), ("reserved", C.c_int32),
                ("tg_u0", C.c_double), ("tg_k", C.c_double), ("tg_nu", C.c_double)]


class BodyState(C.Structure):
    _fields_ = [("step", C.c_int64), ("fx", C.c_double), ("fy", C.c_double),
                ("torque", C.c_double), ("xc", C.c_double), ("yc", C.c_double),
                ("vx", C.c_double), ("vy", C.c_double), ("omega", C.c_double),
                ("slip_mean", C.c_double), ("slip_max", C.c_double),
                ("mdf_residual", C.c_double), ("mdf_omega", C.c_double),
                ("mdf_iters", C.c_int32), ("flags", C.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Launch(C.Structure):
    _fields_ = [("block_x", C.c_int32), ("block_y", C.c_int32), ("rows_per_thread", C.c_int32),
                ("xcd_remap", C.c_int32), ("ib_threads", C.c_int32)]


class ServerConfig(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("precision", C.c_int32), ("hbm_budget", C.c_uint64),
                ("max_resident", C.c_int32), ("quantum", C.c_int32), ("graph_steps", C.c_int32),
                ("spread", C.c_int32), ("launch", Launch), ("stream", C.c_void_p)]


class Request(C.Structure):
    _fields_ = [("lattice", Config), ("n_bodies", C.c_int32), ("bodies", BodyDesc * MAX_BODIES),
                ("steps", C.c_int64), ("rho", C.POINTER(C.c_double)),
                ("ux", C.POINTER(C.c_double)), ("uy", C.POINTER(C.c_double))]


class Result(C.Structure):
    _fields_ = [("id", C.c_int64), ("status", C.c_int32), ("n_bodies", C.c_int32),
                ("steps_done", C.c_int64), ("footprint", C.c_uint64), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_finish", C.c_double),
                ("body", BodyState * MAX_BODIES)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("failed", C.c_int64), ("resident", C.c_int64), ("queued", C.c_int64),
                ("resident_bytes", C.c_uint64), ("peak_resident_bytes", C.c_uint64),
                ("peak_resident", C.c_int64), ("node_updates", C.c_int64), ("rounds", C.c_int64),
                ("busy_seconds", C.c_double), ("now", C.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load ``libib_lbm.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP runtime under the same soname; importing it
    # first makes this library bind to that runtime, so the process holds a
    # single HIP runtime whose streams and memory both sides share.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2609_02298_amd/build.py "
                          "(there is no CPU fallback)")
    L = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    vp = C.c_void_p
    L.ib_lbm_abi_version.restype = C.c_uint32
    L.ib_lbm_create.argtypes = [C.POINTER(Config), C.POINTER(vp)]
    L.ib_lbm_add_body.argtypes = [vp, C.POINTER(BodyDesc), C.POINTER(C.c_int32)]
    L.ib_lbm_step.argtypes = [vp, C.c_int64]
    L.ib_lbm_forces.argtypes = [vp, C.c_int32, C.POINTER(BodyState)]
    L.ib_lbm_history.argtypes = [vp, C.c_int32, C.c_int64, C.c_int64, dp]
    L.ib_lbm_fields.argtypes = [vp, dp, dp, dp]
    L.ib_lbm_get_populations.argtypes = [vp, dp]
    L.ib_lbm_set_populations.argtypes = [vp, dp]
    L.ib_lbm_set_equilibrium.argtypes = [vp, dp, dp, dp]
    L.ib_lbm_force_field.argtypes = [vp, dp, dp]
    L.ib_lbm_markers.argtypes = [vp, C.c_int32, dp, C.POINTER(C.c_int32)]
    L.ib_lbm_diagnostics.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, dp, dp]
    L.ib_lbm_diagnostics_noalloc.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, dp, dp]
    L.ib_lbm_steps_done.argtypes = [vp, C.POINTER(C.c_int64)]
    L.ib_lbm_sync.argtypes = [vp]
    L.ib_lbm_destroy.argtypes = [vp]
    L.ib_lbm_last_error.restype = C.c_char_p
    L.ib_lbm_last_error.argtypes = [vp]
    L.ib_lbm_footprint.restype = C.c_size_t
    L.ib_lbm_footprint.argtypes = [C.POINTER(Config), C.c_int32, C.POINTER(C.c_int32)]
    L.ib_lbm_set_launch.argtypes = [vp, C.POINTER(Launch)]
    L.ib_lbm_get_launch.argtypes = [vp, C.POINTER(Launch)]
    L.ib_lbm_set_spread.argtypes = [vp, C.c_int32]
    L.ib_lbm_set_graph.argtypes = [vp, C.c_int32]
    L.ib_lbm_set_overlap.argtypes = [vp, C.c_int32]
    L.ib_lbm_stream_copy.argtypes = [vp, vp, C.c_size_t, C.c_int32, vp]
    L.ib_lbm_set_fused.argtypes = [vp, C.c_int32]
    L.ib_lbm_get_fused.argtypes = [vp, C.POINTER(C.c_int32)]
    L.ib_lbm_time_collide_stream.argtypes = [vp, C.c_int32, dp, C.POINTER(C.c_int64)]
    L.ib_lbm_get_overlap.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
    L.ib_lbm_timing_enable.argtypes = [vp, C.c_int32]
    L.ib_lbm_timing_read.argtypes = [vp, C.c_int32, dp, C.POINTER(C.c_int64)]
    L.ib_lbm_batch_create.argtypes = [vp, C.c_int32, C.POINTER(vp)]
    L.ib_lbm_batch_attach.argtypes = [vp, vp]
    L.ib_lbm_batch_detach.argtypes = [vp, vp]
    L.ib_lbm_batch_set_target.argtypes = [vp, vp, C.c_int64]
    L.ib_lbm_batch_step.argtypes = [vp, C.c_int64]
    L.ib_lbm_batch_set_graph.argtypes = [vp, C.c_int32]
    L.ib_lbm_batch_sync.argtypes = [vp]
    L.ib_lbm_batch_destroy.argtypes = [vp]
    L.ib_lbm_batch_last_error.restype = C.c_char_p
    L.ib_lbm_batch_last_error.argtypes = [vp]
    L.ib_lbm_batch_set_launch.argtypes = [vp, C.POINTER(Launch)]
    L.ib_lbm_batch_set_spread.argtypes = [vp, C.c_int32]
    L.ib_lbm_server_create.argtypes = [C.POINTER(ServerConfig), C.POINTER(vp)]
    L.ib_lbm_server_submit.argtypes = [vp, C.POINTER(Request), C.POINTER(C.c_int64)]
    L.ib_lbm_server_wait.argtypes = [vp, C.c_int64, C.c_double, C.POINTER(Result)]
    L.ib_lbm_server_stats_get.argtypes = [vp, C.POINTER(ServerStats)]
    L.ib_lbm_server_drain.argtypes = [vp]
    L.ib_lbm_server_destroy.argtypes = [vp]
    L.ib_lbm_server_last_error.restype = C.c_char_p
    L.ib_lbm_server_last_error.argtypes = [vp]
    if L.ib_lbm_abi_version() != ABI_VERSION:
        raise ImportError("libib_lbm.so ABI version mismatch")
    _lib = L
    return L


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _torch_stream(stream):
    if stream is not None:
        return int(stream)
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device available (the library has no CPU path)")
    return int(torch.cuda.current_stream().cuda_stream)


class _TorchAllocator:
    """Routes the library's device allocations through PyTorch's caching
    allocator (so lattices share torch's memory pool)."""

    def __init__(self):
        import torch
        self.torch = torch
        self.device = torch.cuda.current_device()
        self._keep = {}

        def _alloc(ctx, nbytes, stream):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, stream or 0)
                return int(p)
            except Exception:
                return None

        def _free(ctx, ptr, stream):
            if ptr:
                torch.cuda.caching_allocator_delete(int(ptr))

        self.struct = Allocator(None, Allocator._fields_[1][1](_alloc), Allocator._fields_[2][1](_free))


def make_config(case: dict, precision: int = FP64, stream=None, allocator=None,
                history_capacity: int = 0) -> Config:
    c = Config()
    c.abi_version = ABI_VERSION
    c.nx, c.ny = int(case["nx"]), int(case["ny"])
    c.precision = int(precision)
    c.collision = int(case.get("collision", BGK))
    c.history_capacity = int(history_capacity)
    c.tau = float(case["tau"])
    c.trt_magic = float(case.get("trt_magic", 0.25))
    c.cm_s_q = float(case.get("cm_s_q", 1.2))
    c.cm_s_eps = float(case.get("cm_s_eps", 1.4))
    c.rho0 = float(case.get("rho0", 1.0))
    for i, b in enumerate(case.get("bc", (PERIODIC,) * 4)):
        c.bc[i] = int(b)
    c.u_bc = float(case.get("u_bc", 0.0))
    g = case.get("gravity", (0.0, 0.0))
    c.gravity[0], c.gravity[1] = float(g[0]), float(g[1])
    ff = case.get("fluid_force", (0.0, 0.0))
    c.fluid_force[0], c.fluid_force[1] = float(ff[0]), float(ff[1])
    c.stream = stream
    c.alloc = C.pointer(allocator.struct) if allocator is not None else None
    return c


def make_body(b: dict) -> BodyDesc:
    d = BodyDesc()
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


def footprint(case: dict, precision: int = FP64) -> int:
    L = load_library()
    c = make_config(case, precision)
    bodies = case.get("bodies", [])
    nm = (C.c_int32 * max(1, len(bodies)))(*[
        int(b.get("n_markers", 0)) or int(round(math.pi * b["diameter"])) for b in bodies])
    return int(L.ib_lbm_footprint(C.byref(c), len(bodies), nm))


def stream_copy(src, dst, workgroups: int = 0, stream=None):
    """The reference read + write stream (ib_lbm_stream_copy): copies the
    bytes of device tensor `src` into device tensor `dst` of the same size
    on the given (default: current) stream, asynchronously."""
    L = load_library()
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("stream_copy: src and dst sizes differ")
    st = L.ib_lbm_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes,
                              int(workgroups), C.c_void_p(_torch_stream(stream)))
    if st != 0:
        raise IbLbmError(st, "ib_lbm_stream_copy failed")


class Sim:
    """One IB-LBM simulation on the HIP device (the ABI's ``ib_lbm_sim``)."""

    def __init__(self, case: dict, precision: int = FP64, stream=None, torch_allocator: bool = False,
                 history_capacity: int = 0, add_bodies: bool = True):
        self.L = load_library()
        self.case = dict(case)
        self.precision = precision
        self._alloc = _TorchAllocator() if torch_allocator else None
        self.stream = _torch_stream(stream)
        self._cfg = make_config(case, precision, self.stream, self._alloc, history_capacity)
        self.nx, self.ny = self._cfg.nx, self._cfg.ny
        h = C.c_void_p()
        self._check(self.L.ib_lbm_create(C.byref(self._cfg), C.byref(h)), None)
        self.h = h
        self.nmarkers = []
        if add_bodies:
            for b in case.get("bodies", []):
                self.add_body(b)

    def _check(self, st, h=None):
        if st != 0:
            msg = self.L.ib_lbm_last_error(h if h is not None else getattr(self, "h", None))
            raise IbLbmError(st, (msg or b"").decode())

    def close(self):
        if getattr(self, "h", None):
            self.L.ib_lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_body(self, body: dict) -> int:
        d = make_body(body)
        bid = C.c_int32()
        self._check(self.L.ib_lbm_add_body(self.h, C.byref(d), C.byref(bid)), self.h)
        n = C.c_int32()
        self._check(self.L.ib_lbm_markers(self.h, bid.value, None, C.byref(n)), self.h)
        self.nmarkers.append(n.value)
        return bid.value

    def step(self, n: int = 1):
        self._check(self.L.ib_lbm_step(self.h, int(n)), self.h)

    def sync(self):
        self._check(self.L.ib_lbm_sync(self.h), self.h)

    def forces(self, body: int = 0, check: bool = True) -> dict:
        st = BodyState()
        r = self.L.ib_lbm_forces(self.h, body, C.byref(st))
        if check:
            self._check(r, self.h)
        d = st.as_dict()
        d["status"] = r
        return d

    def history(self, body: int, first: int, count: int) -> np.ndarray:
        out = np.zeros((count, 16))
        self._check(self.L.ib_lbm_history(self.h, body, first, count, _dp(out)), self.h)
        return out

    def fields(self):
        r = np.empty((self.ny, self.nx)); ux = np.empty_like(r); uy = np.empty_like(r)
        self._check(self.L.ib_lbm_fields(self.h, _dp(r), _dp(ux), _dp(uy)), self.h)
        return r, ux, uy

    def populations(self) -> np.ndarray:
        f = np.empty((9, self.ny, self.nx))
        self._check(self.L.ib_lbm_get_populations(self.h, _dp(f)), self.h)
        return f

    def set_populations(self, f: np.ndarray):
        f = np.ascontiguousarray(f, np.float64)
        assert f.shape == (9, self.ny, self.nx)
        self._check(self.L.ib_lbm_set_populations(self.h, _dp(f)), self.h)

    def set_equilibrium(self, ux: np.ndarray, uy: np.ndarray, rho: np.ndarray | None = None):
        """Populations = the equilibrium of (rho, u) at every node (rho None:
        rho0), computed on the device."""
        shape = (self.ny, self.nx)
        ux = np.ascontiguousarray(np.broadcast_to(ux, shape), np.float64)
        uy = np.ascontiguousarray(np.broadcast_to(uy, shape), np.float64)
        r = None if rho is None else np.ascontiguousarray(np.broadcast_to(rho, shape), np.float64)
        self._check(self.L.ib_lbm_set_equilibrium(self.h, None if r is None else _dp(r), _dp(ux),
                                                  _dp(uy)), self.h)

    def force(self):
        fx = np.empty((self.ny, self.nx)); fy = np.empty_like(fx)
        self._check(self.L.ib_lbm_force_field(self.h, _dp(fx), _dp(fy)), self.h)
        return fx, fy

    def markers(self, body: int = 0) -> np.ndarray:
        out = np.zeros((self.nmarkers[body], 8))
        n = C.c_int32()
        self._check(self.L.ib_lbm_markers(self.h, body, _dp(out), C.byref(n)), self.h)
        return out

    DIAG_KEYS = ("slip_mean", "slip_max", "phi_leak", "u_inside_mean", "u_inside_max",
                 "n_inside", "dp_mean", "force_mean")

    def diagnostics(self, body: int = 0, kappa: int = 2, u_ref: float = 1.0):
        """Boundary-fidelity diagnostics on the device: (summary dict,
        per-marker n_b x 6 array of slip, dp, |F|, rho, u_n, u_t)."""
        sm = np.zeros(8)
        pm = np.zeros((self.nmarkers[body], 6))
        self._check(self.L.ib_lbm_diagnostics(self.h, int(body), int(kappa), float(u_ref), _dp(sm),
                                               _dp(pm)), self.h)
        return dict(zip(self.DIAG_KEYS, sm.tolist())), pm

    def diagnostics_noalloc(self, body: int = 0, kappa: int = 2, u_ref: float = 1.0):
        """The same through ib_lbm_diagnostics_noalloc (static device staging,
        no device allocation)."""
        sm = np.zeros(8)
        pm = np.zeros((self.nmarkers[body], 6))
        self._check(self.L.ib_lbm_diagnostics_noalloc(self.h, int(body), int(kappa), float(u_ref),
                                                       _dp(sm), _dp(pm)), self.h)
        return dict(zip(self.DIAG_KEYS, sm.tolist())), pm

    @property
    def steps_done(self) -> int:
        v = C.c_int64()
        self._check(self.L.ib_lbm_steps_done(self.h, C.byref(v)), self.h)
        return v.value

    def set_launch(self, block_x=64, block_y=4, rows_per_thread=2, xcd_remap=1, ib_threads=0):
        l = Launch(block_x, block_y, rows_per_thread, xcd_remap, ib_threads)
        self._check(self.L.ib_lbm_set_launch(self.h, C.byref(l)), self.h)

    def get_launch(self) -> dict:
        l = Launch()
        self._check(self.L.ib_lbm_get_launch(self.h, C.byref(l)), self.h)
        return {n: getattr(l, n) for n, _ in Launch._fields_}

    def set_spread(self, mode: int):
        self._check(self.L.ib_lbm_set_spread(self.h, int(mode)), self.h)

    def set_graph(self, steps_per_graph: int):
        self._check(self.L.ib_lbm_set_graph(self.h, int(steps_per_graph)), self.h)

    def set_overlap(self, on: bool):
        self._check(self.L.ib_lbm_set_overlap(self.h, 1 if on else 0), self.h)

    def overlap(self) -> tuple[bool, int]:
        """(split step in use, nodes in the tiles launched before the IB pass)"""
        v = C.c_int32()
        n = C.c_int64()
        self._check(self.L.ib_lbm_get_overlap(self.h, C.byref(v), C.byref(n)), self.h)
        return bool(v.value), n.value

    def set_fused(self, on: bool):
        self._check(self.L.ib_lbm_set_fused(self.h, 1 if on else 0), self.h)

    def fused(self) -> bool:
        """Whether steps run as one fused launch each (after the first step)."""
        v = C.c_int32()
        self._check(self.L.ib_lbm_get_fused(self.h, C.byref(v)), self.h)
        return bool(v.value)

    def timing(self, on: bool):
        self._check(self.L.ib_lbm_timing_enable(self.h, 1 if on else 0), self.h)

    def time_collide_stream(self, launches: int) -> tuple[float, int]:
        """(average microseconds per collide-stream launch, inner nodes per
        launch) over back-to-back launches; advances the populations without
        face closures or IB passes (use a sim made for the measurement)."""
        us = C.c_double()
        n = C.c_int64()
        self._check(self.L.ib_lbm_time_collide_stream(self.h, int(launches), C.byref(us), C.byref(n)),
                    self.h)
        return us.value, n.value

    def timing_read(self, which: int):
        ms = C.c_double(); n = C.c_int64()
        self._check(self.L.ib_lbm_timing_read(self.h, which, C.byref(ms), C.byref(n)), self.h)
        return ms.value, n.value


class Batch:
    """Many sims advanced by shared launches (the ABI's ``ib_lbm_batch``)."""

    def __init__(self, precision: int = FP32_SHIFTED, stream=None):
        self.L = load_library()
        self.stream = _torch_stream(stream)
        h = C.c_void_p()
        st = self.L.ib_lbm_batch_create(self.stream, precision, C.byref(h))
        if st != 0:
            raise IbLbmError(st, "batch creation failed")
        self.h = h
        self.sims = []

    def _check(self, st):
        if st != 0:
            raise IbLbmError(st, (self.L.ib_lbm_batch_last_error(self.h) or b"").decode())

    def attach(self, sim: Sim, target: int | None = None):
        self._check(self.L.ib_lbm_batch_attach(self.h, sim.h))
        self.sims.append(sim)
        if target is not None:
            self.set_target(sim, target)

    def detach(self, sim: Sim):
        self._check(self.L.ib_lbm_batch_detach(self.h, sim.h))
        self.sims.remove(sim)

    def set_target(self, sim: Sim, target: int):
        self._check(self.L.ib_lbm_batch_set_target(self.h, sim.h, int(target)))

    def step(self, n: int):
        self._check(self.L.ib_lbm_batch_step(self.h, int(n)))

    def set_graph(self, steps_per_graph: int):
        self._check(self.L.ib_lbm_batch_set_graph(self.h, int(steps_per_graph)))

    def set_launch(self, block_x=128, block_y=2, rows_per_thread=1, xcd_remap=1, ib_threads=0):
        l = Launch(block_x, block_y, rows_per_thread, xcd_remap, ib_threads)
        self._check(self.L.ib_lbm_batch_set_launch(self.h, C.byref(l)))

    def set_spread(self, mode: int):
        self._check(self.L.ib_lbm_batch_set_spread(self.h, int(mode)))

    def sync(self):
        self._check(self.L.ib_lbm_batch_sync(self.h))

    def close(self):
        if getattr(self, "h", None):
            self.L.ib_lbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request loop with continuous batching (the ABI's ``ib_lbm_server``).

    ``submit`` queues a case and returns its id; ``wait`` returns the result
    as a dict (body states, times on the server clock, optional final
    fields).  The worker thread and every HIP call live in the library."""

    def __init__(self, precision: int = FP32_SHIFTED, hbm_budget: int = 0, max_resident: int = 0,
                 quantum: int = 0, graph_steps: int = 0, spread: int = SPREAD_GATHER,
                 launch: dict | None = None, stream=None):
        self.L = load_library()
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available (the library has no CPU path)")
        torch.cuda.init()
        c = ServerConfig()
        c.abi_version = ABI_VERSION
        c.precision = int(precision)
        c.hbm_budget = int(hbm_budget)
        c.max_resident = int(max_resident)
        c.quantum = int(quantum)
        c.graph_steps = int(graph_steps)
        c.spread = int(spread)
        if launch:
            c.launch = Launch(launch["block_x"], launch["block_y"], launch["rows_per_thread"],
                              launch.get("xcd_remap", 1), launch.get("ib_threads", 0))
        c.stream = stream
        self.precision = int(precision)
        h = C.c_void_p()
        st = self.L.ib_lbm_server_create(C.byref(c), C.byref(h))
        if st != 0:
            raise IbLbmError(st, "server creation failed")
        self.h = h
        self._fields = {}
        self._shape = {}

    def submit(self, case: dict, steps: int, fields: bool = False) -> int:
        bodies = case.get("bodies", [])
        if len(bodies) > MAX_BODIES:
            raise ValueError(f"at most {MAX_BODIES} bodies per request")
        r = Request()
        r.lattice = make_config(case, self.precision)
        r.n_bodies = len(bodies)
        for i, b in enumerate(bodies):
            r.bodies[i] = make_body(b)
        r.steps = int(steps)
        out = None
        if fields:
            ny, nx = int(case["ny"]), int(case["nx"])
            out = tuple(np.empty((ny, nx)) for _ in range(3))
            r.rho, r.ux, r.uy = (_dp(a) for a in out)
        rid = C.c_int64()
        st = self.L.ib_lbm_server_submit(self.h, C.byref(r), C.byref(rid))
        if st != 0:
            raise IbLbmError(st, "submit rejected")
        if out is not None:
            self._fields[rid.value] = out
        return rid.value

    def wait(self, rid: int, timeout: float = -1.0) -> dict | None:
        res = Result()
        st = self.L.ib_lbm_server_wait(self.h, int(rid), float(timeout), C.byref(res))
        if st == PENDING:
            return None
        if st != 0:
            raise IbLbmError(st, "wait failed")
        d = {n: getattr(res, n) for n, _ in Result._fields_ if n != "body"}
        d["bodies"] = [res.body[i].as_dict() for i in range(res.n_bodies)]
        d["latency"] = res.t_finish - res.t_submit
        f = self._fields.pop(int(rid), None)
        if f is not None:
            d["rho"], d["ux"], d["uy"] = f
        return d

    def stats(self) -> dict:
        s = ServerStats()
        st = self.L.ib_lbm_server_stats_get(self.h, C.byref(s))
        if st != 0:
            raise IbLbmError(st, "stats failed")
        return s.as_dict()

    def drain(self):
        self.L.ib_lbm_server_drain(self.h)

    def last_error(self) -> str:
        return (self.L.ib_lbm_server_last_error(self.h) or b"").decode()

    def close(self):
        if getattr(self, "h", None):
            self.L.ib_lbm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
