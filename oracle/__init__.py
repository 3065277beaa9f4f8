"""Python harness around the FP64 CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It loads ``oracle/_build/liborc.so``,
built from ``lbm_oracle.cpp`` by :func:`build`, and shares no code with the
GPU library.

All population arrays are node-major numpy arrays of shape (N, Q) (float64,
or complex128 for the complex-step variants), node n = x + nx*(y + ny*z), the
order numpy gives a C-contiguous [z][y][x] array when it is flattened.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.cpp")
SAN_LIB_PATH = os.path.join(_HERE, "_build", "liborc_san.so")
# ORACLE_LIB selects another build of the oracle (the sanitized one)
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "_build", "liborc.so")
_lib = None
_lock = threading.Lock()


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with g++ (FP64, OpenMP).  Returns the library path.

    sanitize=True builds SAN_LIB_PATH with AddressSanitizer and
    UndefinedBehaviorSanitizer instead (load it with gcc's libasan preloaded
    and ORACLE_LIB pointing at it)."""
    path = SAN_LIB_PATH if sanitize else os.path.join(_HERE, "_build", "liborc.so")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + f".tmp{os.getpid()}"
        opt = (["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"])
        cmd = ["g++", "-std=c++17"] + opt + ["-fopenmp", "-fPIC", "-shared", "-Wall",
                                             "-Wno-unknown-pragmas", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)
    return path


class OrcConfig(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dim", ctypes.c_int32), ("thermal", ctypes.c_int32),
                ("objective", ctypes.c_int32),
                ("tau", ctypes.c_double), ("rho0", ctypes.c_double), ("Re", ctypes.c_double),
                ("L_ref", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("q_brink", ctypes.c_double), ("Pr", ctypes.c_double),
                ("k_ratio", ctypes.c_double), ("q_ramp", ctypes.c_double),
                ("q_w", ctypes.c_double), ("T_in", ctypes.c_double), ("w_dp", ctypes.c_double),
                ("symmetric", ctypes.c_int32 * 3), ("pad", ctypes.c_int32),
                ("inlet_rho", ctypes.c_double), ("beta_max", ctypes.c_double)]


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if "ORACLE_LIB" not in os.environ and (
                not os.path.exists(_LIB_PATH) or
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.orc_create.restype = P
        lib.orc_create.argtypes = [ctypes.POINTER(OrcConfig), P]
        lib.orc_last_error.restype = ctypes.c_char_p
        for name in ("orc_destroy",):
            getattr(lib, name).argtypes = [P]
        for name in ("orc_forward_d", "orc_forward_z"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                          P, P]
        lib.orc_adjoint_d.restype = ctypes.c_int
        lib.orc_adjoint_d.argtypes = [P, P, P, P, P, P, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int, P, P]
        lib.orc_cont_adjoint_d.restype = ctypes.c_int
        lib.orc_cont_adjoint_d.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_int, ctypes.c_int, P, P]
        lib.orc_bc_matrix.argtypes = [P, ctypes.c_int, P]
        lib.orc_bc_matrix_thermal.argtypes = [P, ctypes.c_int, P]
        lib.orc_lattice.argtypes = [P, ctypes.c_int, P, P]
        _lib = lib
        return lib


def _ptr(a):
    if a is None:
        return None
    return ctypes.c_void_p(a.ctypes.data)


class Oracle:
    """The oracle for one problem (a `workloads.Workload` or any object with
    the same attributes)."""

    def __init__(self, w):
        self.lib = _load()
        self.w = w
        cfg = OrcConfig(nx=w.nx, ny=w.ny, nz=w.nz, dim=w.dim, thermal=int(bool(w.thermal)),
                        objective=int(w.objective), tau=w.tau, rho0=w.rho0, Re=w.Re,
                        L_ref=w.L_ref, alpha_max=w.alpha_max, q_brink=w.q_brink, Pr=w.Pr,
                        k_ratio=w.k_ratio, q_ramp=w.q_ramp, q_w=w.q_w, T_in=w.T_in,
                        w_dp=w.w_dp, inlet_rho=float(getattr(w, "inlet_rho", 0.0)),
                        beta_max=float(getattr(w, "beta_max", 0.0)))
        for a, v in enumerate(getattr(w, "symmetric", (0, 0, 0))):
            cfg.symmetric[a] = int(bool(v))
        self._cfg = cfg
        mask = np.ascontiguousarray(w.mask, dtype=np.uint8).reshape(-1)
        self._mask = mask
        h = self.lib.orc_create(ctypes.byref(cfg), _ptr(mask))
        if not h:
            raise ValueError("oracle: " + self.lib.orc_last_error().decode())
        self.h = ctypes.c_void_p(h)
        sizes = np.zeros(6, dtype=np.int32)
        self.lib.orc_sizes(self.h, _ptr(sizes))
        self.N, self.Q, self.Qg, self.n_inlet, self.n_layer, self.n_nonwall = map(int, sizes)
        self.thermal = self.Qg > 0
        self.gamma = np.ascontiguousarray(w.gamma, dtype=np.float64).reshape(-1)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.orc_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # ------------------------------------------------------------------ helpers
    def _g(self, g, dtype=np.float64):
        if self.thermal:
            if g is None:
                return np.zeros((self.N, self.Qg), dtype=dtype)
            return np.ascontiguousarray(g, dtype=dtype)
        return np.zeros((1, 1), dtype=dtype)

    def _gam(self, gamma, dtype=np.float64):
        if gamma is None:
            gamma = self.gamma
        return np.ascontiguousarray(np.asarray(gamma).reshape(-1), dtype=dtype)

    def lattice(self, which: int = 0):
        Q = self.Q if which == 0 else (self.Qg or 7)
        e = np.zeros((Q, 3), dtype=np.int32)
        wt = np.zeros(Q, dtype=np.float64)
        self.lib.orc_lattice(self.h, which, _ptr(e), _ptr(wt))
        return e, wt

    def geometry(self):
        u_in = np.zeros(self.N)
        layer = np.zeros(self.N, dtype=np.uint8)
        self.lib.orc_geometry(self.h, _ptr(u_in), _ptr(layer))
        return u_in, layer

    # ---------------------------------------------------------- forward pieces
    def init(self, complex_: bool = False):
        dt = np.complex128 if complex_ else np.float64
        f = np.zeros((self.N, self.Q), dtype=dt)
        g = self._g(None, dt)
        (self.lib.orc_init_z if complex_ else self.lib.orc_init_d)(self.h, _ptr(f), _ptr(g))
        return f, (g if self.thermal else None)

    def collide(self, f, g=None, gamma=None):
        cz = np.iscomplexobj(f) or np.iscomplexobj(g) or np.iscomplexobj(gamma)
        dt = np.complex128 if cz else np.float64
        f = np.array(f, dtype=dt, order="C", copy=True)
        g = self._g(g, dt).copy()
        gam = self._gam(gamma, dt)
        (self.lib.orc_collide_z if cz else self.lib.orc_collide_d)(self.h, _ptr(gam), _ptr(f),
                                                                 _ptr(g))
        return f, (g if self.thermal else None)

    def stream(self, fC, gC=None):
        cz = np.iscomplexobj(fC) or np.iscomplexobj(gC)
        dt = np.complex128 if cz else np.float64
        fC = np.ascontiguousarray(fC, dtype=dt)
        gC = self._g(gC, dt)
        fS = np.zeros_like(fC)
        gS = np.zeros_like(gC)
        (self.lib.orc_stream_z if cz else self.lib.orc_stream_d)(self.h, _ptr(fC), _ptr(gC),
                                                               _ptr(fS), _ptr(gS))
        return fS, (gS if self.thermal else None)

    def boundary(self, fS, gS=None):
        cz = np.iscomplexobj(fS) or np.iscomplexobj(gS)
        dt = np.complex128 if cz else np.float64
        f = np.array(fS, dtype=dt, order="C", copy=True)
        g = self._g(gS, dt).copy()
        (self.lib.orc_boundary_z if cz else self.lib.orc_boundary_d)(self.h, _ptr(f), _ptr(g))
        return f, (g if self.thermal else None)

    def step(self, f, g=None, gamma=None):
        """One forward step B(S(C(f))) (Eq. 35)."""
        fC, gC = self.collide(f, g, gamma)
        fS, gS = self.stream(fC, gC)
        return self.boundary(fS, gS)

    def forward(self, gamma=None, max_steps=None, tol=None, check_every=None, state=None,
                complex_: bool = False):
        """Forward solve; returns dict(f, g, steps, status, res)."""
        w = self.w
        max_steps = w.max_steps if max_steps is None else max_steps
        tol = w.tol if tol is None else tol
        check_every = w.check_every if check_every is None else check_every
        cz = complex_ or np.iscomplexobj(gamma) or (state is not None and
                                                    np.iscomplexobj(state[0]))
        dt = np.complex128 if cz else np.float64
        gam = self._gam(gamma, dt)
        if state is None:
            f = np.zeros((self.N, self.Q), dtype=dt)
            g = self._g(None, dt)
            warm = 0
        else:
            f = np.array(state[0], dtype=dt, order="C", copy=True)
            g = self._g(state[1], dt).copy()
            warm = 1
        steps = np.zeros(1, dtype=np.int32)
        res = np.zeros(2)
        fn = self.lib.orc_forward_z if cz else self.lib.orc_forward_d
        st = fn(self.h, _ptr(gam), _ptr(f), _ptr(g), int(max_steps), float(tol),
                int(check_every), warm, _ptr(steps), _ptr(res))
        return {"f": f, "g": g if self.thermal else None, "steps": int(steps[0]),
                "status": int(st), "res": res}

    def macro(self, f, g=None):
        """rho [N], u [N,3], T [N] (or None) from a post-boundary state."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        rho = np.zeros(self.N)
        u = np.zeros((self.N, 3))
        T = np.zeros(self.N) if self.thermal else None
        g = self._g(g)
        self.lib.orc_macro_d(self.h, _ptr(f), _ptr(g), _ptr(rho), _ptr(u), _ptr(T))
        return rho, u, T

    def objective(self, f, g=None, gamma=None):
        cz = np.iscomplexobj(f) or np.iscomplexobj(g) or np.iscomplexobj(gamma)
        if cz:
            J = np.zeros(1, dtype=np.complex128)
            self.lib.orc_objective_z(self.h, _ptr(self._gam(gamma, np.complex128)),
                                     _ptr(np.ascontiguousarray(f, dtype=np.complex128)),
                                     _ptr(self._g(g, np.complex128)), _ptr(J))
            return complex(J[0])
        J = np.zeros(1)
        self.lib.orc_objective_d(self.h, _ptr(self._gam(gamma)),
                                 _ptr(np.ascontiguousarray(f, dtype=np.float64)),
                                 _ptr(self._g(g)), _ptr(J))
        return float(J[0])

    def objective_grad(self, f, g=None, gamma=None):
        jf = np.zeros((self.N, self.Q))
        jg = self._g(None)
        jgam = np.zeros(self.N)
        self.lib.orc_objective_grad_d(self.h, _ptr(self._gam(gamma)),
                                      _ptr(np.ascontiguousarray(f, dtype=np.float64)),
                                      _ptr(self._g(g)), _ptr(jf), _ptr(jg), _ptr(jgam))
        return jf, (jg if self.thermal else None), jgam

    def monitor(self, f, g=None):
        out = np.zeros(2)
        self.lib.orc_forward_monitor_d(self.h, _ptr(np.ascontiguousarray(f, dtype=np.float64)),
                                       _ptr(self._g(g)), _ptr(out))
        return out

    # ---------------------------------------------------------- adjoint pieces
    def bc_matrix(self, node: int, thermal: bool = False):
        Q = self.Qg if thermal else self.Q
        B = np.zeros((Q, Q))
        (self.lib.orc_bc_matrix_thermal if thermal else self.lib.orc_bc_matrix)(
            self.h, int(node), _ptr(B))
        return B

    def adjoint_bc(self, fsC, gsC=None):
        fsC = np.ascontiguousarray(fsC, dtype=np.float64)
        gsC = self._g(gsC)
        fs = np.zeros_like(fsC)
        gs = np.zeros_like(gsC)
        self.lib.orc_adjoint_bc_d(self.h, _ptr(fsC), _ptr(gsC), _ptr(fs), _ptr(gs))
        return fs, (gs if self.thermal else None)

    def adjoint_stream(self, fs, gs=None):
        fs = np.ascontiguousarray(fs, dtype=np.float64)
        gs = self._g(gs)
        fsS = np.zeros_like(fs)
        gsS = np.zeros_like(gs)
        self.lib.orc_adjoint_stream_d(self.h, _ptr(fs), _ptr(gs), _ptr(fsS), _ptr(gsS))
        return fsS, (gsS if self.thermal else None)

    def adjoint_collide(self, f, g, fsS, gsS=None, jf=None, jg=None, gamma=None):
        f = np.ascontiguousarray(f, dtype=np.float64)
        fsS = np.ascontiguousarray(fsS, dtype=np.float64)
        jf = np.zeros_like(fsS) if jf is None else np.ascontiguousarray(jf, dtype=np.float64)
        gsS = self._g(gsS)
        jg = self._g(jg)
        fsC = np.zeros_like(fsS)
        gsC = self._g(None)
        self.lib.orc_adjoint_collide_d(self.h, _ptr(self._gam(gamma)), _ptr(f),
                                       _ptr(self._g(g)), _ptr(fsS), _ptr(gsS), _ptr(jf),
                                       _ptr(jg), _ptr(fsC), _ptr(gsC))
        return fsC, (gsC if self.thermal else None)

    def adjoint_step(self, f, g, fsC, gsC=None, jf=None, jg=None, gamma=None):
        """One adjoint step: C^T S^T B^T f*_C - dJ/df (Eqs. 54-56)."""
        fs, gs = self.adjoint_bc(fsC, gsC)
        fsS, gsS = self.adjoint_stream(fs, gs)
        return self.adjoint_collide(f, g, fsS, gsS, jf, jg, gamma)

    def adjoint(self, f, g=None, gamma=None, max_steps=None, tol=None, check_every=None,
                state=None):
        """Adjoint solve from the converged forward state (f, g); returns
        dict(fsC, gsC, steps, status, res)."""
        w = self.w
        max_steps = w.max_steps if max_steps is None else max_steps
        tol = w.tol if tol is None else tol
        check_every = w.check_every if check_every is None else check_every
        if state is None:
            fsC = np.zeros((self.N, self.Q))
            gsC = self._g(None)
            warm = 0
        else:
            fsC = np.array(state[0], dtype=np.float64, order="C", copy=True)
            gsC = self._g(state[1]).copy()
            warm = 1
        steps = np.zeros(1, dtype=np.int32)
        res = np.zeros(2)
        st = self.lib.orc_adjoint_d(self.h, _ptr(self._gam(gamma)),
                                    _ptr(np.ascontiguousarray(f, dtype=np.float64)),
                                    _ptr(self._g(g)), _ptr(fsC), _ptr(gsC), int(max_steps),
                                    float(tol), int(check_every), warm, _ptr(steps), _ptr(res))
        return {"fsC": fsC, "gsC": gsC if self.thermal else None, "steps": int(steps[0]),
                "status": int(st), "res": res}

    # ------------------------------------------------- continuous adjoint (Sec. 2.3)
    def cont_adjoint_bc(self, fsS, jfb=None):
        """Boundary step of the continuous adjoint on streamed values fsS
        [N, Q]; jfb is the boundary part of dJ/df (zero if None)."""
        fsS = np.ascontiguousarray(fsS, dtype=np.float64)
        jfb = np.zeros_like(fsS) if jfb is None else np.ascontiguousarray(jfb, dtype=np.float64)
        out = np.zeros_like(fsS)
        self.lib.orc_cont_adjoint_bc_d(self.h, _ptr(jfb), _ptr(fsS), _ptr(out))
        return out

    def cont_adjoint(self, f, gamma=None, max_steps=None, tol=None, check_every=None,
                     state=None):
        """Continuous adjoint solve (Eqs. 23-30, boundary step generalised from
        Eqs. 25-29) from the converged forward state f; flow lattice only.
        Returns dict(fsB, steps, status, res)."""
        if self.thermal:
            raise ValueError("oracle: the continuous adjoint is for the flow lattice only")
        w = self.w
        max_steps = w.max_steps if max_steps is None else max_steps
        tol = w.tol if tol is None else tol
        check_every = w.check_every if check_every is None else check_every
        if state is None:
            fsB = np.zeros((self.N, self.Q))
            warm = 0
        else:
            fsB = np.array(state, dtype=np.float64, order="C", copy=True)
            warm = 1
        steps = np.zeros(1, dtype=np.int32)
        res = np.zeros(2)
        st = self.lib.orc_cont_adjoint_d(self.h, _ptr(self._gam(gamma)),
                                         _ptr(np.ascontiguousarray(f, dtype=np.float64)),
                                         _ptr(fsB), int(max_steps), float(tol), int(check_every),
                                         warm, _ptr(steps), _ptr(res))
        return {"fsB": fsB, "steps": int(steps[0]), "status": int(st), "res": res}

    def cont_sensitivity(self, f, fsB, gamma=None):
        """dJ/dgamma of the continuous adjoint (Eq. 32 with the exact
        derivative of Eq. 12, as in Eq. 66)."""
        dJ = np.zeros(self.N)
        self.lib.orc_cont_sensitivity_d(self.h, _ptr(self._gam(gamma)),
                                        _ptr(np.ascontiguousarray(f, dtype=np.float64)),
                                        _ptr(np.ascontiguousarray(fsB, dtype=np.float64)),
                                        _ptr(dJ))
        return dJ

    def adjoint_monitor(self, fsS, gsS=None):
        out = np.zeros(2)
        self.lib.orc_adjoint_monitor_d(self.h, _ptr(np.ascontiguousarray(fsS, dtype=np.float64)),
                                       _ptr(self._g(gsS)), _ptr(out))
        return out

    def sens_contract(self, f, g, fsS, gsS=None, gamma=None):
        out = np.zeros(self.N)
        self.lib.orc_sens_contract_d(self.h, _ptr(self._gam(gamma)),
                                     _ptr(np.ascontiguousarray(f, dtype=np.float64)),
                                     _ptr(self._g(g)),
                                     _ptr(np.ascontiguousarray(fsS, dtype=np.float64)),
                                     _ptr(self._g(gsS)), _ptr(out))
        return out

    def sensitivity(self, f, g, fsC, gsC=None, gamma=None):
        """dJ/dgamma (Eq. 66) from the converged forward state and adjoint state."""
        dJ = np.zeros(self.N)
        self.lib.orc_sensitivity_d(self.h, _ptr(self._gam(gamma)),
                                   _ptr(np.ascontiguousarray(f, dtype=np.float64)),
                                   _ptr(self._g(g)),
                                   _ptr(np.ascontiguousarray(fsC, dtype=np.float64)),
                                   _ptr(self._g(gsC)), _ptr(dJ))
        return dJ

    # -------------------------------------------------------------- composite
    def solve(self, gamma=None, fwd_steps=None, adj_steps=None, tol=None, check_every=None):
        """Forward solve, adjoint solve and sensitivity; returns a dict with the
        macroscopic fields, J and dJ/dgamma."""
        fw = self.forward(gamma, max_steps=fwd_steps, tol=tol, check_every=check_every)
        f, g = fw["f"], fw["g"]
        rho, u, T = self.macro(f, g)
        J = self.objective(f, g, gamma)
        if getattr(self.w, "adjoint_kind", 0) == 1:
            ca = self.cont_adjoint(f, gamma, max_steps=adj_steps, tol=tol, check_every=check_every)
            dJ = self.cont_sensitivity(f, ca["fsB"], gamma)
            return {"f": f, "g": g, "rho": rho, "u": u, "T": T, "J": J, "dJ": dJ,
                    "fwd_steps": fw["steps"], "fwd_status": fw["status"],
                    "adj_steps": ca["steps"], "adj_status": ca["status"], "fsB": ca["fsB"]}
        ad = self.adjoint(f, g, gamma, max_steps=adj_steps, tol=tol, check_every=check_every)
        dJ = self.sensitivity(f, g, ad["fsC"], ad["gsC"], gamma)
        return {"f": f, "g": g, "rho": rho, "u": u, "T": T, "J": J, "dJ": dJ,
                "fwd_steps": fw["steps"], "fwd_status": fw["status"],
                "adj_steps": ad["steps"], "adj_status": ad["status"],
                "fsC": ad["fsC"], "gsC": ad["gsC"]}


def set_threads(n: int) -> None:
    """OpenMP threads for oracle calls made from the calling host thread."""
    _load().orc_set_threads(int(n))


def threads_used() -> int:
    """Threads the oracle's OpenMP loops use in this process."""
    n = os.environ.get("OMP_NUM_THREADS")
    if n:
        try:
            return max(1, int(n))
        except ValueError:
            pass
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1
