"""ctypes binding of the C ABI in include/lbmadj.h (argument marshalling only).

Every step of the hot path runs in the gfx950 library ``_build/liblbmadj.so``;
this module only converts torch tensors to device pointers and HIP streams,
and raises :class:`LBMError` on a negative status.  There is no CPU fallback:
importing the binding without the built library raises.

torch is imported first so that the library binds to the HIP runtime torch
already loaded (both use the soname libamdhip64.so.7).
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_int32, c_size_t, c_uint64, c_void_p

import torch

# LBMADJ_LIB selects another build of the library (the host-sanitized one)
LIB_PATH = os.environ.get("LBMADJ_LIB") or os.path.join(
    os.path.dirname(os.path.abspath(__file__)), "_build", "liblbmadj.so")

LBM_OK, LBM_NOT_CONVERGED = 0, 1
LBM_ADJOINT_DISCRETE, LBM_ADJOINT_CONTINUOUS = 0, 1
LBM_EINVAL, LBM_ESTATE, LBM_ENOMEM, LBM_EDEVICE, LBM_EDIVERGED = -1, -2, -3, -4, -5
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "ESTATE", -3: "ENOMEM",
                -4: "EDEVICE", -5: "EDIVERGED"}

LBM_OBJ_PRESSURE_DROP, LBM_OBJ_DISSIPATION, LBM_OBJ_HEATSINK, LBM_OBJ_HEATGEN = 0, 1, 2, 3
STATE_FLOW, STATE_THERMAL, STATE_ADJ_FLOW, STATE_ADJ_THERMAL, STATE_GNEQ = 0, 1, 2, 3, 4


class LBMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class lbm_levelset_info_t(ctypes.Structure):
    _fields_ = [("lambda_", c_double), ("volume", c_double), ("G", c_double),
                ("scale", c_double)]


class lbm_desc_t(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("thermal", c_int32),
                ("periodic", c_int32 * 3), ("objective", c_int32),
                ("tau", c_double), ("rho0", c_double), ("Re", c_double), ("L_ref", c_double),
                ("alpha_max", c_double), ("q_brink", c_double), ("Pr", c_double),
                ("k_ratio", c_double), ("q_ramp", c_double), ("q_w", c_double),
                ("T_in", c_double), ("w_dp", c_double),
                ("max_steps", c_int32), ("check_every", c_int32), ("tol", c_double),
                ("adjoint_kind", c_int32), ("symmetric", c_int32 * 3),
                ("inlet_rho", c_double), ("beta_max", c_double)]


class lbm_info_t(ctypes.Structure):
    _fields_ = [("steps", c_int32), ("status", c_int32), ("residual", c_double * 2),
                ("monitor", c_double * 2), ("J", c_double)]

    def as_dict(self) -> dict:
        return {"steps": int(self.steps), "status": int(self.status),
                "residual": [float(self.residual[0]), float(self.residual[1])],
                "monitor": [float(self.monitor[0]), float(self.monitor[1])], "J": float(self.J)}


class lbm_batch_result_t(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_int64), ("state", c_int32), ("status", c_int32),
                ("nodes", c_int32), ("fwd_steps", c_int32), ("adj_steps", c_int32),
                ("reserved", c_int32), ("J", c_double)]


class lbm_batch_stats_t(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_uint64), ("bytes_in_use", ctypes.c_uint64),
                ("running", c_int32), ("finished", c_int32), ("queued", c_int32),
                ("reserved", c_int32), ("launches", ctypes.c_int64),
                ("node_updates", ctypes.c_int64)]


LBM_BATCH_QUEUED, LBM_BATCH_RUNNING, LBM_BATCH_DONE, LBM_BATCH_FAILED = 0, 1, 2, 3
LBM_BATCH_POLICY_ALL, LBM_BATCH_POLICY_SRW, LBM_BATCH_POLICY_OVERLAP = 0, 1, 2
LBM_BATCH_POLICY_OVERLAP_FIFO = 3

EXPORTS = ("lbm_problem_create", "lbm_workspace_bytes", "lbm_bind_workspace",
           "lbm_bind_static_workspace", "lbm_forward_solve",
           "lbm_forward_continue", "lbm_adjoint_solve", "lbm_adjoint_continue",
           "lbm_thermal_resolve", "lbm_sensitivity", "lbm_forward_resume",
           "lbm_adjoint_resume", "lbm_levelset_update",
           "lbm_copy_state", "lbm_set_kernel_timing", "lbm_kernel_timing", "lbm_stream_probe",
           "lbm_copy_probe",
           "lbm_lattice",
           "lbm_problem_destroy", "lbm_last_error", "lbm_batch_create", "lbm_batch_table_bytes",
           "lbm_batch_bind_arena", "lbm_batch_set_policy", "lbm_batch_set_persistent", "lbm_batch_submit", "lbm_batch_step", "lbm_batch_poll",
           "lbm_batch_stats", "lbm_batch_destroy")

_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblbmadj.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2501_02161_amd.build`"
                          " (there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    P = c_void_p
    lib.lbm_problem_create.argtypes = [POINTER(lbm_desc_t), P, POINTER(c_void_p)]
    lib.lbm_problem_create.restype = c_int
    lib.lbm_workspace_bytes.argtypes = [P]
    lib.lbm_workspace_bytes.restype = c_size_t
    lib.lbm_bind_workspace.argtypes = [P, P, c_size_t]
    lib.lbm_bind_workspace.restype = c_int
    lib.lbm_bind_static_workspace.argtypes = [P]
    lib.lbm_bind_static_workspace.restype = c_int
    lib.lbm_forward_solve.argtypes = [P, P, P, P, P, POINTER(lbm_info_t), P]
    lib.lbm_forward_solve.restype = c_int
    lib.lbm_forward_continue.argtypes = [P, P, c_int32, P, P, P, POINTER(lbm_info_t), P]
    lib.lbm_forward_continue.restype = c_int
    lib.lbm_adjoint_solve.argtypes = [P, P, P, P, P, POINTER(lbm_info_t), P]
    lib.lbm_adjoint_solve.restype = c_int
    lib.lbm_adjoint_continue.argtypes = [P, P, P, P, P, c_int32, POINTER(lbm_info_t), P]
    lib.lbm_adjoint_continue.restype = c_int
    lib.lbm_forward_resume.argtypes = [P, P, P, P, P, POINTER(lbm_info_t), P]
    lib.lbm_forward_resume.restype = c_int
    lib.lbm_adjoint_resume.argtypes = [P, P, P, P, P, POINTER(lbm_info_t), P]
    lib.lbm_adjoint_resume.restype = c_int
    lib.lbm_levelset_update.argtypes = [P, P, P, P, P, c_double, POINTER(c_double), c_double,
                                        POINTER(lbm_levelset_info_t), P]
    lib.lbm_levelset_update.restype = c_int
    lib.lbm_thermal_resolve.argtypes = [P, P, P, P, POINTER(lbm_info_t), P]
    lib.lbm_thermal_resolve.restype = c_int
    lib.lbm_sensitivity.argtypes = [P, P, P, P, P, P, POINTER(c_double), P]
    lib.lbm_sensitivity.restype = c_int
    lib.lbm_copy_state.argtypes = [P, c_int32, P, P]
    lib.lbm_copy_state.restype = c_int
    lib.lbm_set_kernel_timing.argtypes = [P, c_int32]
    lib.lbm_set_kernel_timing.restype = c_int
    lib.lbm_kernel_timing.argtypes = [P, P, P, c_int32]
    lib.lbm_kernel_timing.restype = c_int
    lib.lbm_stream_probe.argtypes = [P, P, c_int32, POINTER(c_double), P]
    lib.lbm_stream_probe.restype = c_int
    lib.lbm_copy_probe.argtypes = [P, P, c_uint64, c_int32, POINTER(c_double), P]
    lib.lbm_copy_probe.restype = c_int
    lib.lbm_lattice.argtypes = [c_int32, P, P]
    lib.lbm_lattice.restype = c_int
    lib.lbm_problem_destroy.argtypes = [P]
    lib.lbm_problem_destroy.restype = None
    lib.lbm_last_error.argtypes = []
    lib.lbm_last_error.restype = c_char_p
    lib.lbm_batch_create.argtypes = [c_int32, c_int32, c_int32, c_int32, POINTER(c_void_p)]
    lib.lbm_batch_create.restype = c_int
    lib.lbm_batch_table_bytes.argtypes = [P, c_size_t]
    lib.lbm_batch_table_bytes.restype = c_size_t
    lib.lbm_batch_bind_arena.argtypes = [P, P, c_size_t]
    lib.lbm_batch_bind_arena.restype = c_int
    lib.lbm_batch_set_policy.argtypes = [P, c_int32, c_int32]
    lib.lbm_batch_set_policy.restype = c_int
    lib.lbm_batch_set_persistent.argtypes = [P, c_int32]
    lib.lbm_batch_set_persistent.restype = c_int
    lib.lbm_batch_submit.argtypes = [P, POINTER(lbm_desc_t), P, P, POINTER(ctypes.c_int64)]
    lib.lbm_batch_submit.restype = c_int
    lib.lbm_batch_step.argtypes = [P, P, POINTER(c_int32), POINTER(c_int32)]
    lib.lbm_batch_step.restype = c_int
    lib.lbm_batch_poll.argtypes = [P, ctypes.c_int64, POINTER(lbm_batch_result_t), P, P]
    lib.lbm_batch_poll.restype = c_int
    lib.lbm_batch_stats.argtypes = [P, POINTER(lbm_batch_stats_t)]
    lib.lbm_batch_stats.restype = c_int
    lib.lbm_batch_destroy.argtypes = [P]
    lib.lbm_batch_destroy.restype = None
    _lib = lib
    return lib


def _check(rc: int) -> int:
    if rc < 0:
        raise LBMError(rc, load_library().lbm_last_error().decode())
    return rc


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return c_void_p(t)
    if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.float32):
        raise ValueError("fields must be contiguous float32 device tensors")
    return c_void_p(t.data_ptr())


def _stream(stream, device=None):
    if stream is None:
        stream = torch.cuda.current_stream(device)
    if isinstance(stream, int):
        return c_void_p(stream)
    return c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------- C names
def lbm_problem_create(desc: lbm_desc_t, mask) -> c_void_p:
    import numpy as np
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    h = c_void_p()
    _check(load_library().lbm_problem_create(byref(desc), c_void_p(m.ctypes.data), byref(h)))
    return h


def lbm_workspace_bytes(p) -> int:
    return int(load_library().lbm_workspace_bytes(p))


def lbm_bind_workspace(p, ws: torch.Tensor) -> None:
    _check(load_library().lbm_bind_workspace(p, c_void_p(ws.data_ptr()), ws.numel()))


def lbm_bind_static_workspace(p) -> None:
    """Bind the library's static workspace of the current device (no device
    allocation; at most 32 MiB; one problem per device owns it at a time)."""
    _check(load_library().lbm_bind_static_workspace(p))


def lbm_forward_solve(p, gamma, drho, u, T, stream=None) -> lbm_info_t:
    info = lbm_info_t()
    _check(load_library().lbm_forward_solve(p, _ptr(gamma), _ptr(drho), _ptr(u), _ptr(T),
                                            byref(info), _stream(stream)))
    return info


def lbm_forward_continue(p, gamma, nsteps, drho, u, T, stream=None) -> lbm_info_t:
    info = lbm_info_t()
    _check(load_library().lbm_forward_continue(p, _ptr(gamma), int(nsteps), _ptr(drho), _ptr(u),
                                               _ptr(T), byref(info), _stream(stream)))
    return info


def lbm_adjoint_solve(p, gamma, drho, u, T, stream=None) -> lbm_info_t:
    info = lbm_info_t()
    _check(load_library().lbm_adjoint_solve(p, _ptr(gamma), _ptr(drho), _ptr(u), _ptr(T),
                                            byref(info), _stream(stream)))
    return info


def lbm_adjoint_continue(p, gamma, drho, u, T, nsteps, stream=None) -> lbm_info_t:
    info = lbm_info_t()
    _check(load_library().lbm_adjoint_continue(p, _ptr(gamma), _ptr(drho), _ptr(u), _ptr(T),
                                               int(nsteps), byref(info), _stream(stream)))
    return info


def lbm_forward_resume(p, gamma, drho, u, T, stream=None) -> lbm_info_t:
    info = lbm_info_t()
    _check(load_library().lbm_forward_resume(p, _ptr(gamma), _ptr(drho), _ptr(u), _ptr(T),
                                             byref(info), _stream(stream)))
    return info


def lbm_adjoint_resume(p, gamma, drho, u, T, stream=None) -> lbm_info_t:
    info = lbm_info_t()
    _check(load_library().lbm_adjoint_resume(p, _ptr(gamma), _ptr(drho), _ptr(u), _ptr(T),
                                             byref(info), _stream(stream)))
    return info


def lbm_levelset_update(p, phi, phi_out, dJ, gamma, K, sigma, vmax, stream=None) -> dict:
    """sigma: a scalar or the per-axis coefficients (sigma_x, sigma_y, sigma_z)."""
    import numpy as np
    info = lbm_levelset_info_t()
    sg = (c_double * 3)(*np.broadcast_to(np.asarray(sigma, dtype=np.float64), (3,)).tolist())
    _check(load_library().lbm_levelset_update(p, _ptr(phi), _ptr(phi_out), _ptr(dJ), _ptr(gamma),
                                              float(K), sg, float(vmax), byref(info),
                                              _stream(stream)))
    return {"lambda": info.lambda_, "volume": info.volume, "G": info.G, "scale": info.scale}


def lbm_thermal_resolve(p, gamma, u, T, stream=None) -> lbm_info_t:
    info = lbm_info_t()
    _check(load_library().lbm_thermal_resolve(p, _ptr(gamma), _ptr(u), _ptr(T), byref(info),
                                              _stream(stream)))
    return info


def lbm_sensitivity(p, gamma, drho, u, T, dJ, stream=None) -> float:
    J = c_double()
    _check(load_library().lbm_sensitivity(p, _ptr(gamma), _ptr(drho), _ptr(u), _ptr(T), _ptr(dJ),
                                          byref(J), _stream(stream)))
    return float(J.value)


def lbm_copy_state(p, which: int, dst, stream=None) -> None:
    _check(load_library().lbm_copy_state(p, int(which), _ptr(dst), _stream(stream)))


def lbm_set_kernel_timing(p, enable: bool) -> None:
    """Bracket every forward / adjoint sweep with HIP events (see the header)."""
    _check(load_library().lbm_set_kernel_timing(p, int(bool(enable))))


def lbm_kernel_timing(p, reset: bool = False):
    """((ms_forward, ms_adjoint), (launches_forward, launches_adjoint))."""
    import numpy as np
    ms = np.zeros(2, dtype=np.float64)
    n = np.zeros(2, dtype=np.int64)
    _check(load_library().lbm_kernel_timing(p, c_void_p(ms.ctypes.data), c_void_p(n.ctypes.data),
                                            int(bool(reset))))
    return (float(ms[0]), float(ms[1])), (int(n[0]), int(n[1]))


def lbm_stream_probe(p, gamma, launches: int, stream=None) -> float:
    """Microseconds per launch of the forward step's traffic without its
    arithmetic (the workspace's states are lost)."""
    us = c_double(0.0)
    _check(load_library().lbm_stream_probe(p, _ptr(gamma), int(launches), byref(us),
                                           _stream(stream, gamma.device)))
    return us.value


def lbm_copy_probe(src: torch.Tensor, dst: torch.Tensor, launches: int, stream=None) -> float:
    """Microseconds per launch of the library's streaming copy of src into
    dst (same size, 16-byte aligned device tensors)."""
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("copy probe buffers must be contiguous device tensors")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("copy probe buffers differ in size")
    us = c_double(0.0)
    _check(load_library().lbm_copy_probe(c_void_p(src.data_ptr()), c_void_p(dst.data_ptr()),
                                         nbytes, int(launches), byref(us),
                                         _stream(stream, src.device)))
    return us.value


def lbm_lattice(which: int):
    import numpy as np
    Q = {0: 19, 1: 7, 2: 9, 3: 5}.get(int(which), 19)
    e = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q, dtype=np.float64)
    _check(load_library().lbm_lattice(int(which), c_void_p(e.ctypes.data),
                                      c_void_p(w.ctypes.data)))
    return e, w


def lbm_problem_destroy(p) -> None:
    load_library().lbm_problem_destroy(p)


def lbm_last_error() -> str:
    return load_library().lbm_last_error().decode()


def lbm_batch_create(thermal: bool, objective: int, max_slots: int, quantum: int) -> c_void_p:
    h = c_void_p()
    _check(load_library().lbm_batch_create(int(bool(thermal)), int(objective), int(max_slots),
                                           int(quantum), byref(h)))
    return h


def lbm_batch_table_bytes(b, arena_bytes: int) -> int:
    return int(load_library().lbm_batch_table_bytes(b, int(arena_bytes)))


def lbm_batch_bind_arena(b, arena: torch.Tensor) -> None:
    _check(load_library().lbm_batch_bind_arena(b, c_void_p(arena.data_ptr()), arena.numel()))


def lbm_batch_set_policy(b, policy: int, fill_tiles: int = 512) -> None:
    _check(load_library().lbm_batch_set_policy(b, int(policy), int(fill_tiles)))


def lbm_batch_set_persistent(b, max_tiles: int) -> None:
    _check(load_library().lbm_batch_set_persistent(b, int(max_tiles)))


def lbm_batch_submit(b, desc: lbm_desc_t, mask, gamma) -> int:
    import numpy as np
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    g = np.ascontiguousarray(gamma, dtype=np.float32).reshape(-1)
    t = ctypes.c_int64()
    _check(load_library().lbm_batch_submit(b, byref(desc), c_void_p(m.ctypes.data),
                                           c_void_p(g.ctypes.data), byref(t)))
    return int(t.value)


def lbm_batch_step(b, stream=None):
    a, q = c_int32(), c_int32()
    _check(load_library().lbm_batch_step(b, _stream(stream), byref(a), byref(q)))
    return int(a.value), int(q.value)


def lbm_batch_poll(b, ticket: int, dJ_host=None, stream=None) -> lbm_batch_result_t:
    r = lbm_batch_result_t()
    ptr = None if dJ_host is None else c_void_p(dJ_host.ctypes.data)
    _check(load_library().lbm_batch_poll(b, int(ticket), byref(r), ptr, _stream(stream)))
    return r


def lbm_batch_stats(b) -> dict:
    st = lbm_batch_stats_t()
    _check(load_library().lbm_batch_stats(b, byref(st)))
    return {k: int(getattr(st, k)) for k, _ in lbm_batch_stats_t._fields_ if k != "reserved"}


def lbm_batch_destroy(b) -> None:
    load_library().lbm_batch_destroy(b)


# ------------------------------------------------------------- convenience
def make_desc(spec) -> lbm_desc_t:
    """lbm_desc_t from any object with the descriptor's attribute names."""
    d = lbm_desc_t()
    d.nx, d.ny, d.nz = int(spec.nx), int(spec.ny), int(spec.nz)
    d.thermal = int(bool(spec.thermal))
    per = getattr(spec, "periodic", (False, False, False))
    for a in range(3):
        d.periodic[a] = int(bool(per[a]))
    d.objective = int(spec.objective)
    for name in ("tau", "rho0", "Re", "L_ref", "alpha_max", "q_brink", "Pr", "k_ratio", "q_ramp",
                 "q_w", "T_in", "w_dp", "tol"):
        setattr(d, name, float(getattr(spec, name)))
    d.max_steps = int(spec.max_steps)
    d.check_every = int(spec.check_every)
    d.adjoint_kind = int(getattr(spec, "adjoint_kind", LBM_ADJOINT_DISCRETE))
    sym = getattr(spec, "symmetric", (False, False, False))
    for a in range(3):
        d.symmetric[a] = int(bool(sym[a]))
    d.inlet_rho = float(getattr(spec, "inlet_rho", 0.0))
    d.beta_max = float(getattr(spec, "beta_max", 0.0))
    return d


class Problem:
    """One lattice problem on one GPU: the C handle plus its bound workspace
    (a torch uint8 tensor) and the output fields as torch tensors."""

    def __init__(self, spec, device=None, static_workspace: bool = False, **overrides):
        self.lib = load_library()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        if overrides:
            spec = spec.replace(**overrides)
        self.spec = spec
        self.desc = make_desc(spec)
        self.h = lbm_problem_create(self.desc, spec.mask)
        self.N = spec.nx * spec.ny * spec.nz
        self.shape = (spec.nz, spec.ny, spec.nx)
        self.thermal = bool(spec.thermal)
        with torch.cuda.device(self.device):
            if static_workspace:
                self.ws = None
                lbm_bind_static_workspace(self.h)
            else:
                self.ws = torch.empty(lbm_workspace_bytes(self.h), dtype=torch.uint8,
                                      device=self.device)
                lbm_bind_workspace(self.h, self.ws)
        z = lambda *s: torch.zeros(*s, dtype=torch.float32, device=self.device)
        self.drho = z(self.shape)
        self.u = z((3,) + self.shape)
        self.T = z(self.shape) if self.thermal else None
        self.dJ = z(self.shape)
        self.fwd_info = None
        self.adj_info = None

    def close(self):
        if getattr(self, "h", None):
            lbm_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def gamma_tensor(self, gamma) -> torch.Tensor:
        if isinstance(gamma, torch.Tensor):
            g = gamma.to(device=self.device, dtype=torch.float32)
        else:
            g = torch.as_tensor(gamma, dtype=torch.float32).to(self.device)
        return g.reshape(self.shape).contiguous()

    def forward(self, gamma, stream=None) -> dict:
        with torch.cuda.device(self.device):
            self._gamma = self.gamma_tensor(gamma)
            self.fwd_info = lbm_forward_solve(self.h, self._gamma, self.drho, self.u, self.T,
                                              stream).as_dict()
        return self.fwd_info

    def forward_continue(self, nsteps: int, stream=None) -> dict:
        with torch.cuda.device(self.device):
            self.fwd_info = lbm_forward_continue(self.h, self._gamma, nsteps, self.drho, self.u,
                                                 self.T, stream).as_dict()
        return self.fwd_info

    def adjoint(self, gamma=None, u=None, T=None, stream=None) -> dict:
        with torch.cuda.device(self.device):
            g = self._gamma if gamma is None else self.gamma_tensor(gamma)
            self._gamma = g
            self.adj_info = lbm_adjoint_solve(self.h, g, None, self.u if u is None else u,
                                              self.T if T is None else T, stream).as_dict()
        return self.adj_info

    def forward_resume(self, gamma=None, stream=None) -> dict:
        """Warm restart of the forward solve (to the residual criterion),
        with a new design field if given."""
        with torch.cuda.device(self.device):
            if gamma is not None:
                self._gamma = self.gamma_tensor(gamma)
            self.fwd_info = lbm_forward_resume(self.h, self._gamma, self.drho, self.u, self.T,
                                               stream).as_dict()
        return self.fwd_info

    def adjoint_resume(self, stream=None) -> dict:
        """Warm restart of the adjoint solve about the current forward state."""
        with torch.cuda.device(self.device):
            self.adj_info = lbm_adjoint_resume(self.h, self._gamma, None, self.u, self.T,
                                               stream).as_dict()
        return self.adj_info

    def adjoint_continue(self, nsteps: int, stream=None) -> dict:
        with torch.cuda.device(self.device):
            self.adj_info = lbm_adjoint_continue(self.h, self._gamma, None, self.u, self.T,
                                                 nsteps, stream).as_dict()
        return self.adj_info

    def sensitivity(self, gamma=None, u=None, T=None, stream=None) -> float:
        with torch.cuda.device(self.device):
            g = self._gamma if gamma is None else self.gamma_tensor(gamma)
            return lbm_sensitivity(self.h, g, None, self.u if u is None else u,
                                   self.T if T is None else T, self.dJ, stream)

    def solve(self, gamma, stream=None) -> dict:
        """Forward solve, adjoint solve and sensitivity."""
        fi = self.forward(gamma, stream)
        ai = self.adjoint(stream=stream)
        J = self.sensitivity(stream=stream)
        return {"forward": fi, "adjoint": ai, "J": J}

    def stream_probe(self, gamma, launches: int = 1000, stream=None) -> float:
        """Microseconds per launch of the forward step's memory traffic with
        none of its arithmetic; every solve state is lost."""
        with torch.cuda.device(self.device):
            return lbm_stream_probe(self.h, self.gamma_tensor(gamma), launches, stream)

    def state(self, which: int) -> torch.Tensor:
        qf, qg = (9, 5) if self.spec.nz == 1 else (19, 7)
        q = qf if which in (STATE_FLOW, STATE_ADJ_FLOW) else qg
        out = torch.empty((q,) + self.shape, dtype=torch.float32, device=self.device)
        with torch.cuda.device(self.device):
            lbm_copy_state(self.h, which, out)
        return out
