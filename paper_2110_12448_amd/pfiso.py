"""Python binding of the C ABI in include/pf.h (libpfiso.so).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch supplies device memory (the solver workspace) and the
stream.  The names mirror the C calls (pf_create, pf_step, pf_read_fields,
pf_tip_state, ...); ``Solver`` wraps them for a problem dictionary as built by
``paper_2110_12448_amd.workloads``.

There is no fallback: if libpfiso.so is missing or fails to load, importing
the library raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpfiso.so")

PF_OK = 0
PF_ERR_ARG = -1
PF_ERR_UNSTABLE_DT = -2
PF_ERR_OOM = -3
PF_ERR_DEVICE = -4
PF_ERR_NONFINITE = -5
PF_ERR_STATE = -6
PF_F32, PF_F64 = 0, 1
PF_BC_NOFLUX, PF_BC_PERIODIC = 0, 1
PF_SCHEME_ISO, PF_SCHEME_STD, PF_SCHEME_WEIGHTS = 0, 1, 2
PF_AT_APPROX, PF_AT_FULL = 0, 1
PF_DIV_SHELLS, PF_DIV_TWO_POINT = 0, 1

EXPORTED = ("pf_version", "pf_last_error", "pf_stable_dt", "pf_workspace_bytes", "pf_create",
            "pf_step", "pf_step_diffusion", "pf_synchronize", "pf_read_fields", "pf_tip_state",
            "pf_tip_fields", "pf_device_fields",
            "pf_frame_state", "pf_tune", "pf_autotune", "pf_geometry", "pf_destroy", "pf_batch_create",
            "pf_batch_step", "pf_batch_use_graph", "pf_batch_autotune", "pf_batch_destroy")


class pf_params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("precision", C.c_int32), ("scheme", C.c_int32), ("weights", C.c_double * 3),
        ("k", C.c_double), ("eps4", C.c_double), ("D", C.c_double), ("lam", C.c_double),
        ("h", C.c_double), ("dt", C.c_double), ("Vp", C.c_double), ("lT", C.c_double),
        ("y0", C.c_double), ("bc", C.c_int32 * 3), ("frame", C.c_int32),
        ("shift_row", C.c_int32), ("n_grains", C.c_int32),
        ("grain_rot", C.POINTER(C.c_double)),
        ("antitrapping", C.c_int32), ("divergence", C.c_int32),
        ("dynamic_grains", C.c_int32),
    ]


class pf_init(C.Structure):
    _fields_ = [("psi", C.POINTER(C.c_double)), ("U", C.POINTER(C.c_double)),
                ("grain", C.POINTER(C.c_int8))]


class pf_tip(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("found", C.c_int32),
                ("nonfinite", C.c_int32), ("index", C.c_int64), ("x", C.c_double),
                ("y_frame", C.c_double), ("z", C.c_double), ("y_lab", C.c_double),
                ("velocity", C.c_double), ("solid_fraction", C.c_double),
                ("frame_shift", C.c_int64)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libpfiso.so.  torch is imported first so that the library binds to
    the HIP runtime torch already holds (same SONAME)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (HIP runtime first)
    if not os.path.exists(path):
        raise ImportError("libpfiso.so not built: run `python -c 'import __graft_entry__ as g; "
                          "g.build()'` (or paper_2110_12448_amd/build.py)")
    lib = C.CDLL(path)
    P = C.POINTER
    lib.pf_version.restype = C.c_int
    lib.pf_last_error.restype = C.c_char_p
    lib.pf_stable_dt.argtypes = [P(pf_params)]
    lib.pf_stable_dt.restype = C.c_double
    lib.pf_workspace_bytes.argtypes = [P(pf_params)]
    lib.pf_workspace_bytes.restype = C.c_size_t
    lib.pf_create.argtypes = [P(pf_params), P(pf_init), C.c_void_p, C.c_size_t, C.c_void_p,
                              P(C.c_void_p)]
    lib.pf_step.argtypes = [C.c_void_p, C.c_int64]
    lib.pf_step_diffusion.argtypes = [C.c_void_p, C.c_int64]
    lib.pf_synchronize.argtypes = [C.c_void_p]
    lib.pf_read_fields.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double), P(C.c_double),
                                   P(C.c_int8)]
    lib.pf_tip_state.argtypes = [C.c_void_p, P(pf_tip)]
    lib.pf_tip_fields.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                  C.c_int32, C.c_double, C.c_int32, C.c_void_p, P(pf_tip)]
    lib.pf_device_fields.argtypes = [C.c_void_p, P(C.c_void_p), P(C.c_void_p)]
    lib.pf_frame_state.argtypes = [C.c_void_p, P(C.c_int64), P(C.c_int32)]
    lib.pf_tune.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
    lib.pf_autotune.argtypes = [C.c_void_p, C.c_int32, P(C.c_int32), P(C.c_int32)]
    lib.pf_geometry.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_int32)]
    lib.pf_destroy.argtypes = [C.c_void_p]
    lib.pf_destroy.restype = None
    lib.pf_batch_create.argtypes = [P(C.c_void_p), C.c_int32, P(C.c_void_p)]
    lib.pf_batch_step.argtypes = [C.c_void_p, C.c_int64]
    lib.pf_batch_use_graph.argtypes = [C.c_void_p, C.c_int32]
    lib.pf_batch_autotune.argtypes = [C.c_void_p, C.c_int32, P(C.c_int32)]
    lib.pf_batch_destroy.argtypes = [C.c_void_p]
    lib.pf_batch_destroy.restype = None
    for name in ("pf_create", "pf_step", "pf_synchronize", "pf_read_fields", "pf_tip_state",
                 "pf_tip_fields",
                 "pf_device_fields", "pf_frame_state", "pf_tune", "pf_autotune",
                 "pf_geometry", "pf_batch_create", "pf_batch_step", "pf_batch_use_graph", "pf_batch_autotune"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


class PFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("pf error %d: %s" % (code, msg))
        self.code = code


def _check(rc: int):
    if rc != PF_OK:
        raise PFError(rc, load().pf_last_error().decode())


def make_params(prob: dict, precision: int = PF_F32, scheme: Optional[int] = None) -> tuple:
    """pf_params from a workloads problem dict; returns (params, keepalive)."""
    rot = np.ascontiguousarray(np.asarray(prob["rot"], dtype=np.float64).reshape(-1, 9))
    p = pf_params()
    p.dim, p.nx, p.ny = int(prob["dim"]), int(prob["nx"]), int(prob["ny"])
    p.nz = int(prob.get("nz", 1)) if p.dim == 3 else 1
    p.precision = int(precision)
    w = tuple(prob["w"])
    if scheme is None:
        p.scheme = PF_SCHEME_WEIGHTS
    else:
        p.scheme = int(scheme)
    for i in range(3):
        p.weights[i] = float(w[i]) if i < len(w) else 0.0
        p.bc[i] = int(prob["bc"][i])
    if p.dim == 2:
        p.weights[2] = 0.0
    p.k, p.eps4, p.D, p.lam = prob["k"], prob["eps4"], prob["D"], prob["lam"]
    p.h, p.dt, p.Vp, p.lT, p.y0 = prob["h"], prob["dt"], prob["Vp"], prob["lT"], prob["y0"]
    p.frame, p.shift_row = int(prob["frame"]), int(prob["shift_row"])
    p.n_grains = rot.shape[0]
    p.grain_rot = rot.ctypes.data_as(C.POINTER(C.c_double))
    p.antitrapping = int(prob.get("antitrapping", PF_AT_APPROX))
    p.divergence = PF_DIV_TWO_POINT if prob.get("two_point", 0) else PF_DIV_SHELLS
    p.dynamic_grains = int(prob.get("dynamic_grains", 0))
    return p, rot


class Solver:
    """One solve resident on a GPU.  Workspace and stream come from torch."""

    def __init__(self, prob: dict, precision: int = PF_F32, device: str = "cuda:0",
                 stream=None, scheme: Optional[int] = None):
        import torch
        lib = load()
        self.prob = prob
        self.precision = precision
        self.params, self._rot = make_params(prob, precision, scheme)
        self.shape = (prob["nz"], prob["ny"], prob["nx"]) if prob["dim"] == 3 else (prob["ny"], prob["nx"])
        self.device = torch.device(device)
        nbytes = lib.pf_workspace_bytes(C.byref(self.params))
        if nbytes == 0:
            raise PFError(PF_ERR_ARG, lib.pf_last_error().decode())
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        psi = np.ascontiguousarray(prob["psi0"], dtype=np.float64)
        U = np.ascontiguousarray(prob["U0"], dtype=np.float64)
        g = prob.get("grain")
        g = None if g is None else np.ascontiguousarray(g, dtype=np.int8)
        ini = pf_init(psi.ctypes.data_as(C.POINTER(C.c_double)),
                      U.ctypes.data_as(C.POINTER(C.c_double)),
                      None if g is None else g.ctypes.data_as(C.POINTER(C.c_int8)))
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.pf_create(C.byref(self.params), C.byref(ini), C.c_void_p(aligned),
                                 C.c_size_t(nbytes), C.c_void_p(self.stream.cuda_stream),
                                 C.byref(h)))
        self.handle = h

    def step(self, nsteps: int = 1):
        _check(load().pf_step(self.handle, int(nsteps)))

    def step_diffusion(self, nsteps: int = 1):
        """U by the diffusion term of Eq. PF_b alone, psi held (pf_step_diffusion)."""
        _check(load().pf_step_diffusion(self.handle, int(nsteps)))

    def synchronize(self):
        _check(load().pf_synchronize(self.handle))

    def read_fields(self):
        """(phi, U, psi, grain) as host numpy arrays in frame coordinates."""
        phi = np.empty(self.shape)
        U = np.empty(self.shape)
        psi = np.empty(self.shape)
        g = np.empty(self.shape, dtype=np.int8)
        dp = C.POINTER(C.c_double)
        _check(load().pf_read_fields(self.handle, phi.ctypes.data_as(dp), U.ctypes.data_as(dp),
                                     psi.ctypes.data_as(dp),
                                     g.ctypes.data_as(C.POINTER(C.c_int8))))
        return phi, U, psi, g

    def tip_state(self, allow_nonfinite: bool = False) -> dict:
        t = pf_tip()
        rc = load().pf_tip_state(self.handle, C.byref(t))
        if rc != PF_OK and not (allow_nonfinite and rc == PF_ERR_NONFINITE):
            _check(rc)
        return {f: getattr(t, f) for f, _ in pf_tip._fields_}

    def tip_fields(self, allow_nonfinite: bool = False) -> dict:
        """pf_tip_fields on this solver's current device fields (the reduction
        without allocation; no solver bookkeeping such as step or velocity)."""
        psi, U = self.device_fields()
        _, pend = self.frame_state()
        t = pf_tip()
        rc = load().pf_tip_fields(C.c_void_p(psi), C.c_void_p(U), self.precision,
                                  self.params.nx, self.params.ny,
                                  self.params.nz if self.params.dim == 3 else 1,
                                  self.params.h, pend, C.c_void_p(self.stream.cuda_stream),
                                  C.byref(t))
        if rc != PF_OK and not (allow_nonfinite and rc == PF_ERR_NONFINITE):
            _check(rc)
        return {f: getattr(t, f) for f, _ in pf_tip._fields_}

    def frame_state(self):
        s, p = C.c_int64(), C.c_int32()
        _check(load().pf_frame_state(self.handle, C.byref(s), C.byref(p)))
        return int(s.value), int(p.value)

    def device_fields(self):
        a, b = C.c_void_p(), C.c_void_p()
        _check(load().pf_device_fields(self.handle, C.byref(a), C.byref(b)))
        return a.value, b.value

    def tune(self, rows_per_segment: int, z_tile: int = 1):
        """Launch geometry: rows per wave segment (4..256), or in 2D -k for k
        waves per SIMD (1..64); z rows per workgroup in 3D."""
        _check(load().pf_tune(self.handle, int(rows_per_segment), int(z_tile)))

    def geometry(self):
        """(rows_per_segment, z_tile) of the step launches in use (negative
        rows_per_segment: -(waves per SIMD), the 2D default)."""
        seg, zt = C.c_int32(), C.c_int32()
        _check(load().pf_geometry(self.handle, C.byref(seg), C.byref(zt)))
        return seg.value, zt.value

    def autotune(self, steps_per_trial: int = 10):
        """Time the candidate launch geometries on a scratch copy of the state
        and keep the fastest; returns (rows_per_segment, z_tile)."""
        seg, zt = C.c_int32(), C.c_int32()
        _check(load().pf_autotune(self.handle, int(steps_per_trial), C.byref(seg), C.byref(zt)))
        return seg.value, zt.value

    def close(self):
        if getattr(self, "handle", None) is not None:
            load().pf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several 2D solvers advanced by one kernel launch per step (pf_batch_*)."""

    def __init__(self, solvers, graph_steps: int = 0):
        lib = load()
        self.solvers = list(solvers)
        arr = (C.c_void_p * len(self.solvers))(*[s.handle.value for s in self.solvers])
        h = C.c_void_p()
        _check(lib.pf_batch_create(arr, len(self.solvers), C.byref(h)))
        self.handle = h
        if graph_steps:
            self.use_graph(graph_steps)

    def use_graph(self, steps_per_graph: int):
        _check(load().pf_batch_use_graph(self.handle, int(steps_per_graph)))

    def step(self, nsteps: int = 1):
        _check(load().pf_batch_step(self.handle, int(nsteps)))

    def autotune(self, steps_per_trial: int = 10):
        """Time candidate segment lengths for the whole batch on scratch copies
        of the members and keep the fastest; returns the rows per segment."""
        seg = C.c_int32()
        _check(load().pf_batch_autotune(self.handle, int(steps_per_trial), C.byref(seg)))
        return seg.value

    def close(self):
        if getattr(self, "handle", None) is not None:
            load().pf_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
