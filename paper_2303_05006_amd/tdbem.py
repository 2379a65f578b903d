"""ctypes binding of libtdbem.so (argument marshalling only).

Every step of the time-domain CFIE path runs in the HIP library; this module
only converts arguments.  Device buffers are torch tensors on the current HIP
device; work is issued on torch's current stream unless one is given.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdbem.so")
_LIB = None

# error codes and enums (mirror include/tdbem.h)
OK, EINVAL, ENOMEM, EHIP, EBREAKDOWN, ENOCONV, EUNSTABLE = 0, -1, -2, -3, -4, -5, -6
MODE_DIRECT, MODE_IFMM = 0, 1
INTERP_LAGRANGE, INTERP_CHI_TIME = 0, 1
FP64, FP32, BF16 = 0, 1, 2
GUESS_EXTRAP, GUESS_LEARNED = 0, 1
CFIE1, CFIE2, CFIE3 = 1, 2, 3
DT2_SPLIT, DT2_KERNEL, DT2_INTERP = 0, 1, 2
SOLVER_DEVICE, SOLVER_HOST = 0, 1
M2L_AUTO, M2L_GENERIC, M2L_FFT, M2L_BF16 = 0, 1, 2, 3
Q_NE, Q_EDGES, Q_LMAX, Q_MT, Q_NEAR_NNZ, Q_NEAR_PAIRS, Q_Z0_NNZ, Q_NCELLS, Q_NILIST, Q_WINDOW, \
    Q_GMRES_ITERS, Q_DEVICE_BYTES, Q_STEP, Q_EDGE_LEAF, Q_SETUP_MS, Q_PHASE_MS, Q_PHASE_COUNT, Q_GUESS_USED, \
    Q_CONFIG, Q_D0_NNZ, Q_UNSTABLE, Q_WINDOWS, Q_TUNED, Q_NEAR_LEAF_BYTES, Q_GRAPHS = range(25)
PHASES = ["near", "gmres", "p2m", "m2m", "m2l", "l2l", "l2p", "other", "m2l_sum"]

EXPORTS = ["tdbem_setup", "tdbem_incident_planewave", "tdbem_potentials", "tdbem_step", "tdbem_march",
           "tdbem_step_noalloc",
           "tdbem_reset",
           "tdbem_checkpoint", "tdbem_restore", "tdbem_query", "tdbem_near_rows", "tdbem_profile", "tdbem_guess_weights", "tdbem_guess_capture",
           "tdbem_guess_grad", "tdbem_guess_adam",
           "tdbem_destroy", "tdbem_last_error"]
GUESS_NFEAT, GUESS_NHIDDEN = 116, 128
GUESS_NPARAMS = 116 * 128 + 128 + 128 * 128 + 128 + 128 + 1


class TdbemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tdbem error {code}: {msg}")
        self.code = code


class _Mesh(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("xyz", ctypes.c_void_p),
                ("n_triangles", ctypes.c_int64), ("tri", ctypes.c_void_p)]


class _Config(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("nt", ctypes.c_int32), ("d", ctypes.c_int32),
                ("eps", ctypes.c_double), ("mu", ctypes.c_double),
                ("theta", ctypes.c_double), ("zeta", ctypes.c_double),
                ("cfie", ctypes.c_int32), ("n_quad", ctypes.c_int32),
                ("p_s", ctypes.c_int32), ("p_t", ctypes.c_int32), ("interp", ctypes.c_int32), ("dt2", ctypes.c_int32),
                ("m2l", ctypes.c_int32),
                ("leaf_max", ctypes.c_int32), ("min_level", ctypes.c_int32), ("mu_window", ctypes.c_int32),
                ("box_widen", ctypes.c_int32), ("causal_guard", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("precision", ctypes.c_int32), ("n_rhs", ctypes.c_int32),
                ("gmres_rtol", ctypes.c_double), ("gmres_maxit", ctypes.c_int32), ("gmres_restart", ctypes.c_int32),
                ("guess", ctypes.c_int32), ("solver", ctypes.c_int32), ("gmres_blocks", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("near_kernel", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("growth_limit", ctypes.c_double), ("stream", ctypes.c_void_p)]


def load():
    """Load the HIP library; raises if it has not been built (no fallback)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2303_05006_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.tdbem_setup.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Config), ctypes.POINTER(P)]
        L.tdbem_incident_planewave.argtypes = [P, P, i32, P]
        L.tdbem_potentials.argtypes = [P, P, i32, P]
        L.tdbem_step.argtypes = [P, P, P]
        L.tdbem_step_noalloc.argtypes = [P, P, P]
        L.tdbem_march.argtypes = [P, P, P, i32, P, P]
        L.tdbem_reset.argtypes = [P]
        L.tdbem_checkpoint.argtypes = [P, P, ctypes.POINTER(ctypes.c_size_t)]
        L.tdbem_restore.argtypes = [P, P, ctypes.c_size_t]
        L.tdbem_query.argtypes = [P, i32, P]
        L.tdbem_near_rows.argtypes = [P, P, i32, i32, P]
        L.tdbem_profile.argtypes = [P, i32]
        L.tdbem_guess_weights.argtypes = [P, P, i64]
        L.tdbem_guess_capture.argtypes = [P, P, P]
        f32 = ctypes.c_float
        L.tdbem_guess_grad.argtypes = [P, P, P, i64, P, P, P]
        L.tdbem_guess_adam.argtypes = [P, P, P, P, i32, f32, f32, f32, f32, P]
        L.tdbem_destroy.argtypes = [P]
        L.tdbem_destroy.restype = None
        L.tdbem_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            L[name].restype = L[name].restype if name in ("tdbem_destroy", "tdbem_last_error") else ctypes.c_int
        _LIB = L
    return _LIB


def _check(rc):
    if rc != OK:
        raise TdbemError(rc, load().tdbem_last_error().decode())


@dataclass
class Config:
    dt: float
    nt: int = 1000
    eps: float = 8.854187817620389e-12
    mu: float = 4e-7 * np.pi
    theta: float = 1.0
    zeta: float = 299792458.0 / 2
    cfie: int = CFIE1
    n_quad: int = 3
    p_s: int = 4
    p_t: int = 4
    interp: int = INTERP_CHI_TIME
    dt2: int = DT2_SPLIT
    m2l: int = M2L_AUTO
    leaf_max: int = 64
    min_level: int = 2
    mu_window: int = 8
    box_widen: int = 0
    causal_guard: int = 0
    mode: int = MODE_IFMM
    precision: int = FP64
    n_rhs: int = 1
    gmres_rtol: float = 1e-8
    gmres_maxit: int = 60
    gmres_restart: int = 32
    guess: int = GUESS_EXTRAP
    solver: int = SOLVER_DEVICE
    gmres_blocks: int = 0
    autotune: int = 0
    near_kernel: int = 0
    graph: int = 0
    growth_limit: float = 0.0


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def guess_grad(params, X, Y, grad, loss, stream=None):
    """Loss gradient of the guess network on a batch (device FP32 tensors)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(load().tdbem_guess_grad(_ptr(params), _ptr(X), _ptr(Y), int(X.shape[0]), _ptr(grad), _ptr(loss),
                                   ctypes.c_void_p(s.cuda_stream)))


def guess_adam(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """One Adam step in place on the guess parameters (device FP32 tensors)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(load().tdbem_guess_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(t), lr, beta1, beta2, eps,
                                   ctypes.c_void_p(s.cuda_stream)))


class Solver:
    """One TDBEM context on the current device."""

    def __init__(self, verts, tris, cfg: Config, stream=None):
        import torch
        L = load()
        self.cfg = cfg
        self._verts = np.ascontiguousarray(verts, dtype=np.float64)
        self._tris = np.ascontiguousarray(tris, dtype=np.int32)
        m = _Mesh(len(self._verts), self._verts.ctypes.data_as(ctypes.c_void_p),
                  len(self._tris), self._tris.ctypes.data_as(ctypes.c_void_p))
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        c = _Config(cfg.dt, cfg.nt, 2, cfg.eps, cfg.mu, cfg.theta, cfg.zeta, cfg.cfie, cfg.n_quad,
                    cfg.p_s, cfg.p_t, cfg.interp, cfg.dt2, cfg.m2l, cfg.leaf_max, cfg.min_level, cfg.mu_window,
                    cfg.box_widen, cfg.causal_guard, cfg.mode, cfg.precision, cfg.n_rhs,
                    cfg.gmres_rtol, cfg.gmres_maxit, cfg.gmres_restart, cfg.guess, cfg.solver, cfg.gmres_blocks,
                    cfg.autotune, cfg.near_kernel, cfg.graph,
                    cfg.growth_limit, ctypes.c_void_p(s.cuda_stream))
        h = ctypes.c_void_p()
        _check(L.tdbem_setup(ctypes.byref(m), ctypes.byref(c), ctypes.byref(h)))
        self._h = h
        self.ne = self.query_i64(Q_NE)

    # -------------------------------------------------------------- queries
    def query_i64(self, key):
        v = ctypes.c_int64()
        _check(load().tdbem_query(self._h, key, ctypes.byref(v)))
        return v.value

    def query_i32(self, key):
        v = ctypes.c_int32()
        _check(load().tdbem_query(self._h, key, ctypes.byref(v)))
        return v.value

    def query_f64(self, key):
        v = ctypes.c_double()
        _check(load().tdbem_query(self._h, key, ctypes.byref(v)))
        return v.value

    def query_array(self, key, n, dtype):
        a = np.zeros(n, dtype=dtype)
        _check(load().tdbem_query(self._h, key, a.ctypes.data_as(ctypes.c_void_p)))
        return a

    def edges(self):
        return self.query_array(Q_EDGES, 2 * self.ne, np.int32).reshape(-1, 2)

    def lmax(self):
        return self.query_i32(Q_LMAX)

    def info(self):
        lm = self.lmax()
        return {"ne": self.ne, "lmax": lm, "Mt": self.query_array(Q_MT, lm + 1, np.int32).tolist(),
                "ncells": self.query_array(Q_NCELLS, lm + 1, np.int32).tolist(),
                "nilist": self.query_array(Q_NILIST, lm + 1, np.int64).tolist(),
                "near_nnz": self.query_i64(Q_NEAR_NNZ), "near_pairs": self.query_i64(Q_NEAR_PAIRS),
                "z0_nnz": self.query_i64(Q_Z0_NNZ), "window": self.query_i32(Q_WINDOW),
                "windows": self.query_array(Q_WINDOWS, lm + 1, np.int32).tolist(),
                "device_bytes": self.query_i64(Q_DEVICE_BYTES), "setup_ms": self.query_f64(Q_SETUP_MS),
                "near_leaf_bytes": self.query_i64(Q_NEAR_LEAF_BYTES)}

    # ----------------------------------------------------------------- work
    def incident(self, pulses, step, V):
        pa = np.ascontiguousarray(np.stack([p.as_array() if hasattr(p, "as_array") else np.asarray(p, float)
                                            for p in pulses]), dtype=np.float64)
        _check(load().tdbem_incident_planewave(self._h, pa.ctypes.data_as(ctypes.c_void_p), int(step), _ptr(V)))

    def step(self, V, J):
        _check(load().tdbem_step(self._h, _ptr(V), _ptr(J)))

    def march(self, V, J, n_steps=None, with_iters=False):
        """tdbem_march: V, J [n_steps][n_rhs][N_e] (or [n_steps][N_e]) device
        tensors; returns (code, per-step codes[, per-step GMRES iterations])."""
        n = V.shape[0] if n_steps is None else n_steps
        st = np.zeros(max(n, 1), dtype=np.int32)
        it = np.zeros(max(n, 1), dtype=np.int32)
        rc = load().tdbem_march(self._h, _ptr(V), _ptr(J), int(n), st.ctypes.data_as(ctypes.c_void_p),
                                it.ctypes.data_as(ctypes.c_void_p))
        if rc not in (OK, ENOCONV, EUNSTABLE):
            _check(rc)
        return (rc, st[:n], it[:n]) if with_iters else (rc, st[:n])

    def step_noalloc(self, V, J):
        """tdbem_step with the solve's workspace in the library's static array."""
        _check(load().tdbem_step_noalloc(self._h, _ptr(V), _ptr(J)))

    def step_rc(self, V, J):
        return load().tdbem_step(self._h, _ptr(V), _ptr(J))

    def potentials(self, hist, n_hist, out):
        _check(load().tdbem_potentials(self._h, _ptr(hist) if n_hist > 0 else None, int(n_hist), _ptr(out)))

    def reset(self):
        _check(load().tdbem_reset(self._h))

    def checkpoint(self):
        """Marching state as bytes (host copy)."""
        n = ctypes.c_size_t(0)
        _check(load().tdbem_checkpoint(self._h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(load().tdbem_checkpoint(self._h, buf, ctypes.byref(n)))
        return buf.raw[:n.value]

    def restore(self, state: bytes):
        buf = ctypes.create_string_buffer(state, len(state))
        _check(load().tdbem_restore(self._h, buf, len(state)))

    def config_in_effect(self):
        c = _Config()
        _check(load().tdbem_query(self._h, Q_CONFIG, ctypes.byref(c)))
        return {name: getattr(c, name) for name, _ in _Config._fields_ if name != "stream"}

    def d0_nnz(self):
        """Non-zero coefficients of the all-pairs discretised problem."""
        return self.query_i64(Q_D0_NNZ)

    def unstable(self):
        return self.query_array(Q_UNSTABLE, self.cfg.n_rhs, np.int32)

    def near_rows(self, rows, G):
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        out = np.zeros((len(rows), self.ne, G))
        _check(load().tdbem_near_rows(self._h, rows.ctypes.data_as(ctypes.c_void_p), len(rows), int(G),
                                      out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def profile(self, enable=True):
        _check(load().tdbem_profile(self._h, 1 if enable else 0))

    def phase_times(self):
        ms = self.query_array(Q_PHASE_MS, len(PHASES), np.float64)
        cnt = self.query_array(Q_PHASE_COUNT, len(PHASES), np.int64)
        return {p: (float(ms[i]), int(cnt[i])) for i, p in enumerate(PHASES)}

    def guess_weights(self, params):
        """Load the learned-guess network (FP32, GUESS_NPARAMS values in the
        order W1 [116][128], b1, W2 [128][128], b2, w3, b3)."""
        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        _check(load().tdbem_guess_weights(self._h, p.ctypes.data_as(ctypes.c_void_p), p.size))

    def guess_capture(self, features=None, aux=None):
        """Capture the guess inputs of the following steps into device tensors
        features [n_rhs][N_e][116] float32 and aux [n_rhs][N_e][2] float64
        (scale, extrapolation); no arguments switches capture off."""
        _check(load().tdbem_guess_capture(self._h, _ptr(features), _ptr(aux)))

    def guess_used(self):
        """(step, rhs) pairs so far whose solve started from the learned guess."""
        return self.query_i64(Q_GUESS_USED)

    def gmres_iters(self):
        return self.query_i32(Q_GMRES_ITERS)

    def close(self):
        if getattr(self, "_h", None):
            load().tdbem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
