"""Python binding of libhipib (the C-ABI in include/hipib.h).

Argument marshalling only: every step of the timestep runs in the HIP kernels
of libhipib.so.  Device arrays are torch tensors (float64, contiguous, on the
current HIP device); host set-up arrays are numpy.  Work is enqueued on torch's
current stream.  There is no fallback: if the library is missing, importing
the context fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhipib.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hipib.h")

OK, E_INVAL, E_NOMEM, E_HIP, E_NOCONV, E_NUMERIC, E_STATE = range(7)
FP64, MIXED = 0, 1
NEO_HOOKEAN, HOLZAPFEL_OGDEN = 0, 1
OP_HELMHOLTZ, OP_POISSON = 0, 1
(TIMER_OFF, TIMER_SMOOTH_FINE_POISSON, TIMER_SMOOTH_FINE_HELMHOLTZ, TIMER_RESID_RESTRICT, TIMER_PROLONG,
 TIMER_LEVEL_DOWN, TIMER_LEVEL_UP, TIMER_SMALL_VCYCLE, TIMER_RESID_NORM, TIMER_CG_DOTS, TIMER_CG_DIR,
 TIMER_CG_UPDATE, TIMER_REDUCE, TIMER_RHS, TIMER_DIVERGENCE, TIMER_PROJECT, TIMER_PACK, TIMER_SPREAD,
 TIMER_INTERP, TIMER_FE_FORCE) = range(20)   # hipib_timer
MAX_MATERIALS = 8


class HipIBError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


N_PHASES = 7
PHASES = ("forces", "rhs", "spread", "helmholtz", "poisson", "project", "interp")


class Stats(C.Structure):
    """hipib_stats."""
    _fields_ = [("steps", C.c_int32), ("cycles_last", C.c_int32 * 4), ("relres_last", C.c_double * 4),
                ("cycles_mean", C.c_double * 4), ("timed_steps", C.c_int32),
                ("phase_ms", C.c_double * N_PHASES), ("J_min", C.c_double), ("J_max", C.c_double),
                ("volume", C.c_double), ("kinetic_energy", C.c_double), ("momentum", C.c_double * 3),
                ("max_abs_div", C.c_double)]

    def as_dict(self):
        return {"steps": self.steps, "cycles_last": list(self.cycles_last),
                "relres_last": list(self.relres_last), "cycles_mean": list(self.cycles_mean),
                "timed_steps": self.timed_steps,
                "phase_ms": dict(zip(PHASES, list(self.phase_ms))),
                "J_min": self.J_min, "J_max": self.J_max, "volume": self.volume,
                "kinetic_energy": self.kinetic_energy, "momentum": list(self.momentum),
                "max_abs_div": self.max_abs_div}


class Config(C.Structure):
    _fields_ = [("n", C.c_int32), ("rho", C.c_double), ("mu", C.c_double), ("dt", C.c_double),
                ("mg_pre", C.c_int32), ("mg_post", C.c_int32), ("mg_max_cycles", C.c_int32),
                ("mg_fixed_cycles", C.c_int32), ("mg_coarse_sweeps", C.c_int32),
                ("mg_rtol", C.c_double), ("convection", C.c_int32), ("precision", C.c_int32),
                ("deterministic", C.c_int32), ("mg_krylov", C.c_int32), ("walls", C.c_int32)]


_lib = None


def exported_names():
    """Function names declared by include/hipib.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hipib_[a-z0-9_]+)\s*\(", txt)))


def lib():
    """Loads libhipib.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                              "(or python paper_2503_22695_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        P, i32, f64 = C.c_void_p, C.c_int32, C.c_double
        st = C.c_int
        sig = {
            "hipib_default_config": (None, [P]),
            "hipib_create": (st, [P, P, P]),
            "hipib_destroy": (st, [P]),
            "hipib_set_stream": (st, [P, P]),
            "hipib_last_error": (C.c_char_p, []),
            "hipib_set_mesh": (st, [P, i32, P, i32, P, P, P]),
            "hipib_set_mesh_elements": (st, [P, i32, P, i32, i32, P, P, P]),
            "hipib_set_material": (st, [P, i32, i32, P, i32]),
            "hipib_set_pressure_faces": (st, [P, i32, P]),
            "hipib_set_sheets": (st, [P, i32, P]),
            "hipib_set_tethers": (st, [P, i32, P, P, P]),
            "hipib_set_active_tension": (st, [P, f64]),
            "hipib_active_tension": (f64, [f64, f64, f64, f64]),
            "hipib_set_active_waveform": (st, [P, f64, f64, f64]),
            "hipib_fe_force": (st, [P, P, f64, P]),
            "hipib_spread": (st, [P, P, P, P]),
            "hipib_spread_noalloc": (st, [i32, i32, P, P, P, P]),
            "hipib_get_stats": (st, [P, P, P, P]),
            "hipib_set_phase_timing": (st, [P, i32]),
            "hipib_cavity_pressure": (f64, [f64, f64, f64]),
            "hipib_interpolate": (st, [P, P, P, P]),
            "hipib_mg_solve": (st, [P, i32, i32, P, P, P, P]),
            "hipib_ns_step": (st, [P, P, P, P]),
            "hipib_ib_step": (st, [P, P, P, P, f64]),
            "hipib_advance": (st, [P, P, P, P, f64, i32, f64, f64]),
            "hipib_get_step_stats": (i32, [P, P, P, i32]),
            "hipib_adjoint_step": (st, [P, P, P, P, f64, P, P, P]),
            "hipib_adjoint_reset": (st, [P]),
            "hipib_fe_hvp": (st, [P, P, P, P]),
            "hipib_fe_param_vjp": (st, [P, P, P, P]),
            "hipib_spread_vjp_X": (st, [P, P, P, P, P]),
            "hipib_interp_vjp_X": (st, [P, P, P, P, P]),
            "hipib_convection_vjp": (st, [P, P, P, P]),
            "hipib_timer_enable": (st, [P, i32]),
            "hipib_timer_read": (st, [P, P, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def default_config(**over) -> Config:
    cfg = Config()
    lib().hipib_default_config(C.byref(cfg))
    for k, v in over.items():
        if not hasattr(cfg, k):
            raise KeyError(k)
        setattr(cfg, k, v)
    return cfg


def _check(status: int, where: str):
    if status != OK:
        msg = lib().hipib_last_error()
        raise HipIBError(status, where, msg.decode() if msg else "")


def _dev(t, shape=None, name="array"):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


def _stream_ptr():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """One grid plus (optionally) one Lagrangian mesh on the current HIP device."""

    def __init__(self, cfg: Config):
        self._h = C.c_void_p()
        self.cfg = cfg
        _check(lib().hipib_create(C.byref(cfg), _stream_ptr(), C.byref(self._h)), "hipib_create")
        self.n = cfg.n
        self.n_nodes = 0

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if self._h:
            lib().hipib_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync_stream(self):
        _check(lib().hipib_set_stream(self._h, _stream_ptr()), "hipib_set_stream")

    # -- set-up (host arrays) ---------------------------------------------
    def set_mesh(self, X_ref, conn, fibre, mat_id):
        """conn [n_elems, 8] hexes, [n_elems, 4] P1 or [n_elems, 10] P2 tetrahedra."""
        X_ref = np.ascontiguousarray(X_ref, dtype=np.float64).reshape(-1, 3)
        conn = np.asarray(conn)
        npe = int(conn.shape[1]) if conn.ndim == 2 else 8
        conn = np.ascontiguousarray(conn, dtype=np.int32).reshape(-1, npe)
        fibre = np.ascontiguousarray(fibre, dtype=np.float64).reshape(-1, 3)
        mat_id = np.ascontiguousarray(mat_id, dtype=np.int32).reshape(-1)
        if fibre.shape[0] != conn.shape[0] or mat_id.shape[0] != conn.shape[0]:
            raise ValueError("fibre / mat_id must have one row per element")
        _check(lib().hipib_set_mesh_elements(self._h, X_ref.shape[0], X_ref.ctypes.data,
                                             conn.shape[0], npe, conn.ctypes.data,
                                             fibre.ctypes.data, mat_id.ctypes.data),
               "hipib_set_mesh_elements")
        self.n_nodes = X_ref.shape[0]

    def set_material(self, mat_id: int, model: int, params):
        p = np.ascontiguousarray(params, dtype=np.float64)
        _check(lib().hipib_set_material(self._h, mat_id, model, p.ctypes.data, p.size),
               "hipib_set_material")

    def set_pressure_faces(self, faces):
        f = np.ascontiguousarray(faces, dtype=np.int32).reshape(-1, 4)
        _check(lib().hipib_set_pressure_faces(self._h, f.shape[0], f.ctypes.data),
               "hipib_set_pressure_faces")

    def set_sheets(self, sheet):
        s = np.ascontiguousarray(sheet, dtype=np.float64).reshape(-1, 3)
        _check(lib().hipib_set_sheets(self._h, s.shape[0], s.ctypes.data), "hipib_set_sheets")

    def set_tethers(self, node, target, K):
        node = np.ascontiguousarray(node, dtype=np.int32).reshape(-1)
        target = np.ascontiguousarray(target, dtype=np.float64).reshape(-1, 3)
        K = np.ascontiguousarray(K, dtype=np.float64).reshape(-1, 6)
        if target.shape[0] != node.size or K.shape[0] != node.size:
            raise ValueError("tether arrays must have one row per tethered node")
        _check(lib().hipib_set_tethers(self._h, node.size, node.ctypes.data, target.ctypes.data,
                                       K.ctypes.data), "hipib_set_tethers")

    def set_active_tension(self, Ta: float):
        _check(lib().hipib_set_active_tension(self._h, float(Ta)), "hipib_set_active_tension")

    def set_active_waveform(self, ta_max: float, t_on: float, duration: float):
        _check(lib().hipib_set_active_waveform(self._h, float(ta_max), float(t_on), float(duration)),
               "hipib_set_active_waveform")

    # -- hot path (device tensors) ----------------------------------------
    def _grid_shape(self, comps):
        n = self.n
        return (comps, n, n, n) if comps else (n, n, n)

    def fe_force(self, X, pressure: float = 0.0, F=None):
        import torch
        if F is None:
            F = torch.empty_like(X)
        _check(lib().hipib_fe_force(self._h, _dev(X, (self.n_nodes, 3), "X"), float(pressure),
                                    _dev(F, (self.n_nodes, 3), "F")), "hipib_fe_force")
        return F

    def spread(self, X, F, f):
        _check(lib().hipib_spread(self._h, _dev(X, (self.n_nodes, 3), "X"),
                                  _dev(F, (self.n_nodes, 3), "F"), _dev(f, self._grid_shape(3), "f")),
               "hipib_spread")
        return f

    def interpolate(self, X, u, U=None):
        import torch
        if U is None:
            U = torch.empty_like(X)
        _check(lib().hipib_interpolate(self._h, _dev(X, (self.n_nodes, 3), "X"),
                                       _dev(u, self._grid_shape(3), "u"),
                                       _dev(U, (self.n_nodes, 3), "U")), "hipib_interpolate")
        return U

    def mg_solve(self, op: int, b, x) -> Tuple[np.ndarray, np.ndarray]:
        ncomp = 1 if b.dim() == 3 else b.shape[0]
        shape = self._grid_shape(0 if b.dim() == 3 else ncomp)
        cyc = np.zeros(ncomp, dtype=np.int32)
        rr = np.zeros(ncomp, dtype=np.float64)
        _check(lib().hipib_mg_solve(self._h, op, ncomp, _dev(b, shape, "b"), _dev(x, shape, "x"),
                                    cyc.ctypes.data, rr.ctypes.data), "hipib_mg_solve")
        return cyc, rr

    def ns_step(self, f, u, p):
        fp = C.c_void_p(0) if f is None else _dev(f, self._grid_shape(3), "f")
        _check(lib().hipib_ns_step(self._h, fp, _dev(u, self._grid_shape(3), "u"),
                                   _dev(p, self._grid_shape(0), "p")), "hipib_ns_step")

    def ib_step(self, u, p, X, pressure: float = 0.0):
        _check(lib().hipib_ib_step(self._h, _dev(u, self._grid_shape(3), "u"),
                                   _dev(p, self._grid_shape(0), "p"),
                                   _dev(X, (self.n_nodes, 3), "X"), float(pressure)), "hipib_ib_step")

    def advance(self, u, p, X, t0: float, n_steps: int, p0: float = 0.0, T: float = 0.0):
        _check(lib().hipib_advance(self._h, _dev(u, self._grid_shape(3), "u"),
                                   _dev(p, self._grid_shape(0), "p"),
                                   _dev(X, (self.n_nodes, 3), "X"), float(t0), int(n_steps),
                                   float(p0), float(T)), "hipib_advance")

    # -- discrete adjoint ---------------------------------------------------
    def adjoint_step(self, u_n, X_n, u_np1, pressure, lam_u, lam_X, dtheta):
        """Reverse of one ib_step: lam_u, lam_X in/out; dtheta [8, 4] += (device)."""
        g3, nn = self._grid_shape(3), (self.n_nodes, 3)
        _check(lib().hipib_adjoint_step(self._h, _dev(u_n, g3, "u_n"), _dev(X_n, nn, "X_n"),
                                        _dev(u_np1, g3, "u_np1"), float(pressure),
                                        _dev(lam_u, g3, "lam_u"), _dev(lam_X, nn, "lam_X"),
                                        _dev(dtheta, (MAX_MATERIALS, 4), "dtheta")),
               "hipib_adjoint_step")

    def adjoint_reset(self):
        """Zero the starting points of the reverse step's adjoint solves."""
        _check(lib().hipib_adjoint_reset(self._h), "hipib_adjoint_reset")

    def fe_hvp(self, X, V, HV=None):
        import torch
        if HV is None:
            HV = torch.empty_like(X)
        nn = (self.n_nodes, 3)
        _check(lib().hipib_fe_hvp(self._h, _dev(X, nn, "X"), _dev(V, nn, "V"), _dev(HV, nn, "HV")),
               "hipib_fe_hvp")
        return HV

    def fe_param_vjp(self, X, lamF, dtheta):
        nn = (self.n_nodes, 3)
        _check(lib().hipib_fe_param_vjp(self._h, _dev(X, nn, "X"), _dev(lamF, nn, "lamF"),
                                        _dev(dtheta, (MAX_MATERIALS, 4), "dtheta")),
               "hipib_fe_param_vjp")
        return dtheta

    def spread_vjp_X(self, X, F, lam_f, lamX):
        nn = (self.n_nodes, 3)
        _check(lib().hipib_spread_vjp_X(self._h, _dev(X, nn, "X"), _dev(F, nn, "F"),
                                        _dev(lam_f, self._grid_shape(3), "lam_f"),
                                        _dev(lamX, nn, "lamX")), "hipib_spread_vjp_X")
        return lamX

    def interp_vjp_X(self, X, u, lamU, lamX):
        nn = (self.n_nodes, 3)
        _check(lib().hipib_interp_vjp_X(self._h, _dev(X, nn, "X"), _dev(u, self._grid_shape(3), "u"),
                                        _dev(lamU, nn, "lamU"), _dev(lamX, nn, "lamX")),
               "hipib_interp_vjp_X")
        return lamX

    def convection_vjp(self, u, lam, out=None):
        import torch
        if out is None:
            out = torch.empty_like(u)
        g3 = self._grid_shape(3)
        _check(lib().hipib_convection_vjp(self._h, _dev(u, g3, "u"), _dev(lam, g3, "lam"),
                                          _dev(out, g3, "out")), "hipib_convection_vjp")
        return out

    def timer_enable(self, which: int):
        _check(lib().hipib_timer_enable(self._h, which), "hipib_timer_enable")

    def timer_read(self):
        """(launches, total_ms, algorithmic bytes per launch) since the last read."""
        k, ms, by = C.c_int32(0), C.c_double(0.0), C.c_double(0.0)
        _check(lib().hipib_timer_read(self._h, C.byref(k), C.byref(ms), C.byref(by)),
               "hipib_timer_read")
        return k.value, ms.value, by.value

    def get_stats(self, u=None, X=None) -> dict:
        """hipib_get_stats: step records, phase times, and the diagnostics of u
        ([3, n, n, n]) and X ([n_nodes, 3]) when given."""
        st = Stats()
        up = C.c_void_p(0) if u is None else _dev(u, self._grid_shape(3), "u")
        Xp = C.c_void_p(0) if X is None else _dev(X, (self.n_nodes, 3), "X")
        _check(lib().hipib_get_stats(self._h, up, Xp, C.byref(st)), "hipib_get_stats")
        return st.as_dict()

    def set_phase_timing(self, enable: bool):
        _check(lib().hipib_set_phase_timing(self._h, 1 if enable else 0), "hipib_set_phase_timing")

    def step_stats(self, max_steps: int = 100000):
        cyc = np.zeros((max_steps, 4), dtype=np.int32)
        rr = np.zeros((max_steps, 4), dtype=np.float64)
        k = lib().hipib_get_step_stats(self._h, cyc.ctypes.data, rr.ctypes.data, max_steps)
        return cyc[:k], rr[:k]


def config_for_problem(prob, **over) -> Config:
    kw = dict(n=prob.n, rho=prob.rho, mu=prob.mu, dt=prob.dt, mg_pre=prob.mg_pre,
              mg_post=prob.mg_post, mg_max_cycles=prob.mg_max_cycles, mg_rtol=prob.mg_rtol,
              convection=prob.convection, precision=MIXED if prob.precision == "mixed" else FP64,
              mg_krylov=prob.mg_krylov, walls=prob.walls)
    kw.update(over)
    return default_config(**kw)


def context_for_problem(prob, **over) -> Context:
    """A context holding the problem's grid, mesh, materials and pressure faces."""
    ctx = Context(config_for_problem(prob, **over))
    ctx.set_mesh(prob.X_ref, prob.conn, prob.fibre, prob.mat_id)
    for m, mat in enumerate(prob.materials):
        ctx.set_material(m, mat.model, mat.params)
    if prob.n_faces:
        ctx.set_pressure_faces(prob.faces)
    if prob.sheet is not None:
        ctx.set_sheets(prob.sheet)
    if prob.tethers is not None:
        ctx.set_tethers(*prob.tethers)
    if prob.ta_max:
        ctx.set_active_waveform(prob.ta_max, prob.ta_t_on, prob.ta_duration)
    return ctx


def spread_noalloc(n: int, X, F, f):
    """f += S(X) F on the periodic n^3 grid (FP64), hipib_spread_noalloc: no
    context, no allocation; X, F [n_nodes, 3] and f [3, n, n, n] device float64,
    on the current stream."""
    nn = int(X.shape[0]) if X.dim() == 2 else 0
    _check(lib().hipib_spread_noalloc(int(n), nn, _dev(X, (nn, 3), "X"), _dev(F, (nn, 3), "F"),
                                      _dev(f, (3, n, n, n), "f"), _stream_ptr()),
           "hipib_spread_noalloc")


def cavity_pressure(p0: float, T: float, t: float) -> float:
    """p0 sin^2(pi t / T) as hipib_advance applies it (hipib_cavity_pressure)."""
    return lib().hipib_cavity_pressure(float(p0), float(T), float(t))


def active_tension(ta_max: float, t_on: float, duration: float, t: float) -> float:
    """T_a(t) of the activation waveform (hipib_active_tension)."""
    return lib().hipib_active_tension(float(ta_max), float(t_on), float(duration), float(t))


class Simulation:
    """Device state (u, p, X) of one workload plus its context."""

    def __init__(self, prob, **over):
        import torch
        self.prob = prob
        self.ctx = context_for_problem(prob, **over)
        dev = torch.device("cuda", torch.cuda.current_device())
        self.u = torch.tensor(prob.initial_velocity(), dtype=torch.float64, device=dev).contiguous()
        self.p = torch.zeros((prob.n,) * 3, dtype=torch.float64, device=dev)
        self.X = torch.tensor(prob.X0, dtype=torch.float64, device=dev).contiguous()
        self.t = 0.0

    def advance(self, n_steps: int):
        self.ctx.advance(self.u, self.p, self.X, self.t, n_steps, self.prob.p0, self.prob.T)
        self.t += n_steps * self.prob.dt
        return self


# ---------------------------------------------------------------------------
# differentiable rollout
# ---------------------------------------------------------------------------

class Rollout:
    """n_steps immersed-boundary steps of a workload from (u0, X0) at time t0,
    with the Holzapfel-Ogden parameters (a, b, a_f, b_f) of material `mat`
    as inputs; the backward pass runs the discrete adjoint, recomputing each
    segment of `checkpoint_every` steps from a stored (u, p, X) checkpoint."""

    def __init__(self, prob, n_steps=None, checkpoint_every=10, mat=0, t0=0.0, overlap=True,
                 **cfg_over):
        import torch
        self.prob = prob
        self.cfg_over = cfg_over
        self.ctx = context_for_problem(prob, **cfg_over)
        # overlap: the backward pass recomputes the next segment on a second
        # context and stream, from a worker thread, while the current segment's
        # adjoint steps run (both are latency-bound at moderate grid sizes)
        self.overlap = overlap
        self._rctx = None
        self._rstream = None
        self.n_steps = prob.n_steps if n_steps is None else int(n_steps)
        self.k = max(1, int(checkpoint_every))
        self.mat = mat
        self.t0 = t0
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.u0 = torch.tensor(prob.initial_velocity(), dtype=torch.float64, device=self.dev)
        self.kappa = float(prob.materials[mat].params[4])
        self.sheet_params = [float(v) for v in prob.materials[mat].params[5:]]
        self.last_tape = None

    def pressure(self, s0: int, i: int) -> float:
        """Cavity pressure at step s0 + i, with the time rounded exactly as
        hipib_advance rounds it when called at the start of step s0."""
        t = (self.t0 + s0 * self.prob.dt) + i * self.prob.dt
        return cavity_pressure(self.prob.p0, self.prob.T, t)

    def active(self, s0: int, i: int) -> float:
        """Active tension at step s0 + i, timed like pressure()."""
        t = (self.t0 + s0 * self.prob.dt) + i * self.prob.dt
        return active_tension(self.prob.ta_max, self.prob.ta_t_on, self.prob.ta_duration, t)

    def _material(self, th):
        return th[:4] + [self.kappa] + self.sheet_params

    def set_theta(self, theta):
        th = [float(v) for v in theta.detach().cpu().reshape(-1)]
        self._theta = th
        self.ctx.set_material(self.mat, HOLZAPFEL_OGDEN, self._material(th))

    def forward(self, theta, X0, keep_checkpoints=True):
        """X^N from X0.  With keep_checkpoints, (u, p, X) is stored at the start
        of every segment, and the states of the last segment are kept whole as
        they are computed, so the backward pass recomputes every segment but
        the last.  The stored states and theta form a RolloutTape, kept as
        `last_tape` (and passed to backward by IBRollout); a forward pass
        without checkpoints leaves `last_tape` as it was."""
        import torch
        self.set_theta(theta)
        u = self.u0.clone()
        p = torch.zeros((self.prob.n,) * 3, dtype=torch.float64, device=self.dev)
        X = X0.detach().to(self.dev, torch.float64).contiguous().clone()
        tape = RolloutTape(self._theta) if keep_checkpoints else None
        s = 0
        while s < self.n_steps:
            m = min(self.k, self.n_steps - s)
            if keep_checkpoints and s + m == self.n_steps:
                tape.tail = (s, self._run_segment(u, p, X, s, m))
                u, X = tape.tail[1][0][-1], tape.tail[1][1][-1]
            else:
                if keep_checkpoints:
                    tape.checkpoints.append((s, u.clone(), p.clone(), X.clone()))
                self.ctx.advance(u, p, X, self.t0 + s * self.prob.dt, m, self.prob.p0, self.prob.T)
            s += m
        if keep_checkpoints:
            self.last_tape = tape
            return X.clone()
        return X

    def _run_segment(self, u, p, X, s0, m):
        """m steps from (u, p, X) at step s0 (not modified); every u and X."""
        return self._run_segment_on(self.ctx, u, p, X, s0, m)

    def _reverse_segment(self, s0, us, Xs, lam_u, lam_X, dtheta):
        for i in range(len(us) - 2, -1, -1):
            self.ctx.set_active_tension(self.active(s0, i))
            self.ctx.adjoint_step(us[i], Xs[i], us[i + 1], self.pressure(s0, i), lam_u, lam_X, dtheta)

    def _recompute(self, seg):
        """Worker-thread body: the segment's states on the second context."""
        import torch
        s0, uc, pc, Xc = seg
        with torch.cuda.stream(self._rstream):
            self._rstream.wait_stream(self._main_stream)   # checkpoints are written on the main stream
            out = self._run_segment_on(self._rctx, uc, pc, Xc, s0, min(self.k, self.n_steps - s0))
        self._rstream.synchronize()
        return out

    def _run_segment_on(self, ctx, u, p, X, s0, m):
        us, Xs = [u.clone()], [X.clone()]
        u, p, X = u.clone(), p.clone(), X.clone()
        for i in range(m):
            ctx.set_active_tension(self.active(s0, i))
            ctx.ib_step(u, p, X, self.pressure(s0, i))
            us.append(u.clone())
            Xs.append(X.clone())
        return us, Xs

    def backward(self, grad_XN, tape=None):
        """dL/dtheta, dL/dX0 and dL/du0 from dL/dX^N, through the states of
        `tape` (default: the latest forward pass with checkpoints).  The tape is
        not consumed: the same pass can be reversed again."""
        import torch
        tape = self.last_tape if tape is None else tape
        if tape is None:
            raise RuntimeError("Rollout.backward: no forward pass with checkpoints to reverse")
        lam_X = grad_XN.detach().to(self.dev, torch.float64).contiguous().clone()
        lam_u = torch.zeros_like(self.u0)
        dtheta = torch.zeros((MAX_MATERIALS, 4), dtype=torch.float64, device=self.dev)
        # the adjoint steps and the recomputed segments use the tape's material,
        # whatever forward passes ran since, and the adjoint solves start from
        # zero, whatever backward passes ran before
        self.set_theta(torch.tensor(tape.theta, dtype=torch.float64))
        self.ctx.adjoint_reset()
        segs = list(reversed(tape.checkpoints))
        pending = None
        if self.overlap and segs:
            from concurrent.futures import ThreadPoolExecutor
            self._main_stream = torch.cuda.current_stream()
            if self._rctx is None:
                self._rstream = torch.cuda.Stream()          # default priority
                with torch.cuda.stream(self._rstream):
                    self._rctx = context_for_problem(self.prob, **self.cfg_over)
            self._rctx.set_material(self.mat, HOLZAPFEL_OGDEN, self._material(tape.theta))
            pool = ThreadPoolExecutor(max_workers=1)
            pending = pool.submit(self._recompute, segs[0])
        try:
            if tape.tail is not None:
                s0, (us, Xs) = tape.tail
                self._reverse_segment(s0, us, Xs, lam_u, lam_X, dtheta)
            for idx, (s0, uc, pc, Xc) in enumerate(segs):
                if pending is not None:
                    us, Xs = pending.result()
                    pending = pool.submit(self._recompute, segs[idx + 1]) if idx + 1 < len(segs) else None
                else:
                    us, Xs = self._run_segment(uc, pc, Xc, s0, min(self.k, self.n_steps - s0))
                self._reverse_segment(s0, us, Xs, lam_u, lam_X, dtheta)
        finally:
            if self.overlap and segs:
                if pending is not None:
                    pending.result()
                pool.shutdown(wait=True)
        return dtheta[self.mat].clone(), lam_X, lam_u


class RolloutTape:
    """What one forward pass of a Rollout leaves for its backward pass: the
    material parameters, the checkpoints (step, u, p, X) at the start of every
    segment but the last, and the last segment's states (step, (us, Xs))."""

    def __init__(self, theta):
        self.theta = list(theta)
        self.checkpoints = []
        self.tail = None


def _ibrollout_class():
    import torch

    class IBRollout(torch.autograd.Function):
        """X^N = IBRollout.apply(theta, X0, rollout): differentiable in the four
        Holzapfel-Ogden parameters theta (float64, shape [4]) and the initial
        node positions X0 ([n_nodes, 3], device float64)."""

        @staticmethod
        def forward(fctx, theta, X0, rollout):
            XN = rollout.forward(theta, X0)
            fctx.rollout = rollout
            fctx.tape = rollout.last_tape     # this call's states, whatever runs next
            fctx.theta_device = theta.device
            return XN

        @staticmethod
        def backward(fctx, grad_XN):
            dth, dX0, _ = fctx.rollout.backward(grad_XN.contiguous(), fctx.tape)
            return dth.to(fctx.theta_device), dX0, None

    return IBRollout


_IBR = None


def IBRollout():
    """The torch.autograd.Function class (created on first use so importing this
    module does not require torch)."""
    global _IBR
    if _IBR is None:
        _IBR = _ibrollout_class()
    return _IBR
