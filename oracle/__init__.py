"""Plain FP64 CPU oracle for the stochastic Camassa-Holm particle filter
(Cotter, Crisan & Singh, arXiv 2402.06927).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code with
the GPU library (``paper_2402_06927_amd``) and never imports it.

The numerical work lives in ``sch_oracle.c`` (plain C, ``-O2
-ffp-contract=off``); this module builds it with gcc and wraps it with ctypes
over numpy arrays.  Each wrapper names the C function it calls; the paper
passages are cited there.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sch_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

ORC_OK = 0
ORC_E_ARG = -1
ORC_E_SINGULAR = -2
ORC_E_NONCONVERGED = -3
ORC_E_NONFINITE = -4
ORC_E_DEGENERATE = -5

TAG_INIT, TAG_FORECAST, TAG_PCN, TAG_ACCEPT, TAG_RESAMPLE, TAG_OBS, TAG_NUDGE = range(7)


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (plain C, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "sch_oracle.h"))
    ):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = [
        "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11",
        "-Wall", "-Wextra", "-Wno-unused-parameter", "-shared", "-fPIC",
        _SRC, "-o", tmp, "-lm",
    ]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_u32p = C.POINTER(C.c_uint32)


class OrcModel(C.Structure):
    _fields_ = [
        ("L", C.c_double), ("alpha", C.c_double), ("mu", C.c_double), ("dt", C.c_double),
        ("nx", C.c_int32), ("n_modes", C.c_int32), ("xi", _dp),
        ("picard_tol", C.c_double), ("picard_max", C.c_int32),
    ]


class OrcLbfgsOpts(C.Structure):
    _fields_ = [("gtol", C.c_double), ("max_iter", C.c_int32), ("mem", C.c_int32),
                ("max_back", C.c_int32)]


OBJECTIVE = C.CFUNCTYPE(C.c_int, C.c_void_p, _dp, _dp, _dp)


class OrcRng(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("cycle", C.c_uint32), ("temper_k", C.c_uint32)]


class OrcMatern(C.Structure):
    _fields_ = [("kappa", C.c_double), ("eta", C.c_double), ("k", C.c_int32)]


class OrcCycleStats(C.Structure):
    _fields_ = [
        ("ess", C.c_double), ("resampled", C.c_int32), ("n_temper", C.c_int32),
        ("picard_iters", C.c_int64), ("n_accept", C.c_int64), ("status", C.c_int32),
    ]


def _declare(L):
    sig = {
        "orc_philox4x32_10": (None, [_u32p, C.c_uint64, _u32p]),
        "orc_u01": (C.c_double, [C.c_uint32, C.c_uint32]),
        "orc_normal_pair": (None, [C.c_uint64] + [C.c_uint32] * 4 + [_dp]),
        "orc_uniform": (C.c_double, [C.c_uint64] + [C.c_uint32] * 4),
        "orc_draw_increments": (None, [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_uint32,
                                       C.c_uint32, C.c_uint32, C.c_double, _dp]),
        "orc_draw_increments_rows": (None, [C.c_uint64, C.c_int32, C.c_int32, C.c_int32,
                                            C.c_int32, C.c_uint32, C.c_uint32, C.c_uint32,
                                            C.c_double, _dp]),
        "orc_dense_solve": (C.c_int, [C.c_int32, _dp, _dp, _dp]),
        "orc_tridiag_pivot_solve": (C.c_int, [C.c_int32, C.c_int32, _dp, _dp, _dp, _dp]),
        "orc_cyclic_solve": (C.c_int, [C.c_int32, _dp, _dp, _dp, _dp, _dp]),
        "orc_apply_mass": (None, [C.c_int32, C.c_double, _dp, _dp]),
        "orc_apply_stiff": (None, [C.c_int32, C.c_double, _dp, _dp]),
        "orc_apply_advect": (None, [C.c_int32, _dp, _dp, _dp]),
        "orc_velocity_from_momentum": (C.c_int, [C.POINTER(OrcModel), _dp, _dp]),
        "orc_momentum_from_velocity": (C.c_int, [C.POINTER(OrcModel), _dp, _dp]),
        "orc_step": (C.c_int, [C.POINTER(OrcModel), _dp, _dp, _dp, _dp, _ip]),
        "orc_window": (C.c_int, [C.POINTER(OrcModel), C.c_int32, _dp, _dp, _dp, _dp, _ip]),
        "orc_ensemble_window": (C.c_int, [C.POINTER(OrcModel), C.c_int32, C.c_int32, _dp, _dp,
                                          _dp, _dp, _ip, _ip, C.c_int32]),
        "orc_observe": (None, [C.c_int32, C.c_int32, _dp, _dp]),
        "orc_nll": (C.c_double, [C.c_int32, C.c_int32, _dp, _dp, _dp]),
        "orc_ensemble_nll": (None, [C.c_int32, C.c_int32, C.c_int32, _dp, _dp, _dp, _dp]),
        "orc_weights": (C.c_double, [C.c_int32, _dp, _dp, C.c_double, _dp, _dp]),
        "orc_temper": (C.c_int, [C.c_int32, _dp, C.c_double, C.c_double, C.c_int32, _dp, _dp,
                                 _dp]),
        "orc_resample_systematic": (C.c_int, [C.c_int32, _dp, C.c_double, _ip]),
        "orc_resample_textbook": (C.c_int, [C.c_int32, _dp, C.c_double, _ip]),
        "orc_pcn_accept": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_double]),
        "orc_pcn_linear_chain": (C.c_int64, [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, _dp, _dp,
                                             C.c_double, C.c_double, C.c_double, C.c_double,
                                             C.c_int32, _dp, _dp]),
        "orc_jitter_pcn": (C.c_int, [C.POINTER(OrcModel), C.c_int32, _dp, _dp, C.POINTER(OrcRng),
                                     C.c_int32, C.c_int32, _dp, _dp, _dp, _dp, _dp, _dp,
                                     C.c_double, C.c_double, C.c_int32, _ip, C.c_int32]),
        "orc_bootstrap_cycle": (C.c_int, [C.POINTER(OrcModel), C.c_int32, _dp, _dp, C.c_uint64,
                                          C.c_uint32, C.c_int32, C.c_int32, C.c_double, _dp, _dp,
                                          _dp, C.POINTER(OrcCycleStats), C.c_int32]),
        "orc_bootstrap_cycle_matern": (C.c_int, [C.POINTER(OrcModel), C.POINTER(OrcMatern),
                                                 C.c_int32, _dp, _dp, C.c_uint64, C.c_uint32,
                                                 C.c_int32, C.c_int32, C.c_double, _dp, _dp, _dp,
                                                 C.POINTER(OrcCycleStats), C.c_int32]),
        "orc_tempered_cycle": (C.c_int, [C.POINTER(OrcModel), C.c_int32, _dp, _dp, C.c_uint64,
                                         C.c_uint32, C.c_int32, C.c_int32, C.c_double, C.c_int32,
                                         C.c_double, C.c_int32, C.c_int32, _dp, _dp,
                                         C.POINTER(OrcCycleStats), C.c_int32]),
        "orc_tempered_cycle_linear": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, _dp,
                                                _dp, _dp, _dp, C.c_double, C.c_double, C.c_uint64,
                                                C.c_uint32, C.c_int32, C.c_double, C.c_int32,
                                                C.c_double, C.c_int32, C.c_int32, _dp,
                                                C.POINTER(OrcCycleStats), C.c_int32]),
        "orc_nudge_objective": (C.c_int, [C.POINTER(OrcModel), C.c_int32, _dp, _dp, C.c_int32,
                                          _dp, _dp, _dp, _dp, _dp]),
        "orc_nudge_grad": (C.c_int, [C.POINTER(OrcModel), C.c_int32, _dp, _dp, C.c_int32, _dp,
                                     _dp, _dp, _dp, _dp, _dp]),
        "orc_nudge_grad_tangent": (C.c_int, [C.POINTER(OrcModel), C.c_int32, _dp, _dp, C.c_int32,
                                             _dp, _dp, _dp, _dp, _dp]),
        "orc_lbfgs": (C.c_int, [C.c_int32, OBJECTIVE, C.c_void_p, _dp, C.c_double, C.c_double,
                                C.c_int32, C.c_int32, C.c_int32, _dp, _ip, _ip]),
        "orc_nudge_ensemble": (C.c_int, [C.POINTER(OrcModel), C.c_int32, _dp, _dp, C.c_int32,
                                         C.c_int32, _dp, _dp, _dp, _dp, C.POINTER(OrcLbfgsOpts),
                                         _dp, _ip, _ip, _ip, _ip, C.c_int32]),
        "orc_nudged_potential": (C.c_double, [C.c_double, C.c_int32, C.c_double, _dp, _dp]),
        "orc_step_field": (C.c_int, [C.POINTER(OrcModel), _dp, _dp, _dp, _ip]),
        "orc_pcnl_log_ratio": (C.c_double, [C.c_int32, _dp, C.c_double, _dp, _dp, C.c_double,
                                            _dp, C.c_double, C.c_double, C.c_double]),
        "orc_pcnl_linear_chain": (C.c_int64, [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, _dp,
                                              _dp, C.c_double, C.c_double, C.c_double,
                                              C.c_double, C.c_int32, _dp, _dp]),
        "orc_jitter_pcnl": (C.c_int, [C.POINTER(OrcModel), C.c_int32, _dp, _dp, C.POINTER(OrcRng),
                                      C.c_int32, C.c_int32, _dp, _dp, _dp, _dp, _dp, _dp,
                                      C.c_double, C.c_double, C.c_int32, _ip, C.c_int32]),
        "orc_tempered_cycle_pcnl": (C.c_int, [C.POINTER(OrcModel), C.c_int32, _dp, _dp, C.c_uint64,
                                              C.c_uint32, C.c_int32, C.c_int32, C.c_double,
                                              C.c_int32, C.c_double, C.c_int32, C.c_int32, _dp,
                                              _dp, C.POINTER(OrcCycleStats), C.c_int32]),
        "orc_hmc_trajectory_linear": (None, [C.c_int32, C.c_int32, _dp, _dp, C.c_double,
                                             C.c_double, C.c_double, C.c_int32, C.c_double,
                                             _dp, _dp]),
        "orc_hmc_linear_chain": (C.c_int64, [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, _dp,
                                             _dp, C.c_double, C.c_double, C.c_double, C.c_int32,
                                             C.c_double, C.c_int32, _dp, _dp, C.c_int32]),
        "orc_jitter_hmc": (C.c_int, [C.POINTER(OrcModel), C.c_int32, _dp, _dp, C.POINTER(OrcRng),
                                     C.c_int32, C.c_int32, _dp, _dp, _dp, _dp, _dp, _dp,
                                     C.c_double, C.c_double, C.c_int32, C.c_int32, _ip,
                                     C.c_int32]),
        "orc_tempered_cycle_hmc": (C.c_int, [C.POINTER(OrcModel), C.c_int32, _dp, _dp, C.c_uint64,
                                             C.c_uint32, C.c_int32, C.c_int32, C.c_double,
                                             C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                             C.c_int32, _dp, _dp, C.POINTER(OrcCycleStats),
                                             C.c_int32]),
        "orc_matern_transpose": (C.c_int, [C.c_int32, C.c_double, C.POINTER(OrcMatern), _dp,
                                           _dp]),
        "orc_nudge_grad_matern": (C.c_int, [C.POINTER(OrcModel), C.POINTER(OrcMatern), C.c_int32,
                                            _dp, _dp, C.c_int32, _dp, _dp, _dp, _dp,
                                            C.POINTER(C.c_double), _dp]),
        "orc_nudge_ensemble_matern": (C.c_int, [C.POINTER(OrcModel), C.POINTER(OrcMatern),
                                                C.c_int32, _dp, _dp, C.c_int32, C.c_int32, _dp,
                                                _dp, _dp, _dp, C.POINTER(OrcLbfgsOpts), _dp, _ip,
                                                _ip, _ip, _ip, C.c_int32]),
        "orc_paper_init_from": (C.c_int, [C.c_int32, C.c_double, _dp, C.c_double, C.c_double,
                                          _dp]),
        "orc_paper_init": (C.c_int, [C.c_int32, C.c_double, C.c_uint64, C.c_int32, C.c_int32,
                                     _dp]),
        "orc_ensemble_stats": (None, [C.c_int32, C.c_int32, _dp, _dp, _dp]),
        "orc_matern_field": (C.c_int, [C.c_int32, C.c_double, C.POINTER(OrcMatern), _dp, _dp]),
        "orc_window_matern": (C.c_int, [C.POINTER(OrcModel), C.POINTER(OrcMatern), C.c_int32,
                                        _dp, _dp, _dp, _ip]),
        "orc_ensemble_window_matern": (C.c_int, [C.POINTER(OrcModel), C.POINTER(OrcMatern),
                                                 C.c_int32, C.c_int32, _dp, _dp, _dp, _ip, _ip,
                                                 C.c_int32]),
        "orc_jitter_pcn_matern": (C.c_int, [C.POINTER(OrcModel), C.POINTER(OrcMatern), C.c_int32,
                                            _dp, _dp, C.POINTER(OrcRng), C.c_int32, C.c_int32,
                                            _dp, _dp, _dp, _dp, _dp, _dp, C.c_double, C.c_double,
                                            C.c_int32, _ip, C.c_int32]),
        "orc_tempered_cycle_matern": (C.c_int, [C.POINTER(OrcModel), C.POINTER(OrcMatern),
                                                C.c_int32, _dp, _dp, C.c_uint64, C.c_uint32,
                                                C.c_int32, C.c_int32, C.c_double, C.c_int32,
                                                C.c_double, C.c_int32, C.c_int32, _dp, _dp, _dp,
                                                _dp, _dp, _dp, C.POINTER(OrcCycleStats),
                                                C.c_int32]),
        "orc_jitter_pcn_ctrl": (C.c_int, [C.POINTER(OrcModel), C.c_int32, _dp, _dp,
                                          C.POINTER(OrcRng), C.c_int32, C.c_int32, _dp, _dp, _dp,
                                          _dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_int32,
                                          _ip, C.c_int32]),
        "orc_pcn_linear_chain_ctrl": (C.c_int64, [C.c_uint64, C.c_int32, C.c_int32, C.c_int32,
                                                  _dp, _dp, C.c_double, C.c_double, C.c_double,
                                                  C.c_double, _dp, C.c_int32, _dp, _dp]),
        "orc_nudged_cycle": (C.c_int, [C.POINTER(OrcModel), C.c_int32, _dp, _dp, C.c_uint64,
                                       C.c_uint32, C.c_int32, C.c_int32, C.c_double, C.c_int32,
                                       C.c_double, C.c_int32, C.c_int32, C.POINTER(OrcLbfgsOpts),
                                       _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                       C.POINTER(OrcCycleStats), C.c_int32]),
        "orc_nudged_cycle_warm": (C.c_int, [C.POINTER(OrcModel), C.c_int32, _dp, _dp,
                                            C.c_uint64, C.c_uint32, C.c_int32, C.c_int32,
                                            C.c_double, C.c_int32, C.c_double, C.c_int32,
                                            C.c_int32, C.POINTER(OrcLbfgsOpts), _dp, _ip, _dp,
                                            _dp, _dp, _dp, _dp, _dp, _dp,
                                            C.POINTER(OrcCycleStats), C.c_int32]),
        "orc_jitter_pcn_matern_ctrl": (C.c_int, [C.POINTER(OrcModel), C.POINTER(OrcMatern),
                                                 C.c_int32, _dp, _dp, C.POINTER(OrcRng),
                                                 C.c_int32, C.c_int32, _dp, _dp, _dp, _dp, _dp,
                                                 _dp, _dp, C.c_double, C.c_double, C.c_int32,
                                                 _ip, C.c_int32]),
        "orc_nudged_cycle_matern": (C.c_int, [C.POINTER(OrcModel), C.POINTER(OrcMatern),
                                              C.c_int32, _dp, _dp, C.c_uint64, C.c_uint32,
                                              C.c_int32, C.c_int32, C.c_double, C.c_int32,
                                              C.c_double, C.c_int32, C.c_int32,
                                              C.POINTER(OrcLbfgsOpts), _dp, _dp, _dp, _dp, _dp,
                                              _dp, _dp, C.POINTER(OrcCycleStats), C.c_int32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _d(a):
    """Pointer to a C-contiguous float64 numpy array (None passes NULL)."""
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "need C-contiguous float64"
    return a.ctypes.data_as(_dp)


def _i(a):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def n_threads_default() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# --------------------------------------------------------------------------- RNG
def philox4x32_10(ctr, seed: int) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    out = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, C.c_uint64(seed), out)
    return np.array(list(out), dtype=np.uint32)


def u01(hi: int, lo: int) -> float:
    return lib().orc_u01(hi, lo)


def normal_pair(seed, c0, c1, c2, c3):
    z = np.zeros(2)
    lib().orc_normal_pair(seed, c0, c1, c2, c3, _d(z))
    return z


def uniform(seed, c0, c1, c2, c3) -> float:
    return lib().orc_uniform(seed, c0, c1, c2, c3)


def draw_increments(seed, n_particles, n_steps, n_modes, step0, tag, word3, dt):
    out = np.zeros((n_particles, n_steps, n_modes))
    lib().orc_draw_increments(seed, n_particles, n_steps, n_modes, step0, tag, word3, dt, _d(out))
    return out


def draw_increments_rows(seed, p0, n_particles, n_steps, n_modes, step0, tag, word3, dt):
    """Rows p0 .. p0 + n_particles - 1 of draw_increments."""
    out = np.zeros((n_particles, n_steps, n_modes))
    lib().orc_draw_increments_rows(seed, p0, n_particles, n_steps, n_modes, step0, tag, word3, dt,
                                   _d(out))
    return out


# --------------------------------------------------------------------------- model
@dataclass
class Model:
    """Physical and numerical parameters of the SCH model (section 2)."""
    L: float
    alpha: float
    mu: float
    dt: float
    xi: np.ndarray  # [n_modes][nx]
    picard_tol: float = 1e-13
    picard_max: int = 50

    @property
    def nx(self) -> int:
        return int(self.xi.shape[1])

    @property
    def n_modes(self) -> int:
        return int(self.xi.shape[0])

    @property
    def h(self) -> float:
        return self.L / self.nx

    def c(self) -> OrcModel:
        self._xi = _f64(self.xi)
        return OrcModel(self.L, self.alpha, self.mu, self.dt, self.nx, self.n_modes,
                        _d(self._xi), self.picard_tol, self.picard_max)


def dense_solve(A, b):
    A = _f64(A)
    b = _f64(b)
    x = np.zeros_like(b)
    st = lib().orc_dense_solve(len(b), _d(A), _d(b), _d(x))
    return st, x


def tridiag_pivot_solve(dl, d, du, b):
    b = np.array(b, dtype=np.float64, copy=True, order="C")
    nrhs = 1 if b.ndim == 1 else b.shape[0]
    n = len(d)
    st = lib().orc_tridiag_pivot_solve(n, nrhs, _d(_f64(dl)), _d(_f64(d)), _d(_f64(du)), _d(b))
    return st, b


def cyclic_solve(a, b, c, d):
    x = np.zeros(len(b))
    st = lib().orc_cyclic_solve(len(b), _d(_f64(a)), _d(_f64(b)), _d(_f64(c)), _d(_f64(d)),
                                _d(x))
    return st, x


def apply_mass(h, f):
    f = _f64(f)
    out = np.zeros_like(f)
    lib().orc_apply_mass(len(f), h, _d(f), _d(out))
    return out


def apply_stiff(h, f):
    f = _f64(f)
    out = np.zeros_like(f)
    lib().orc_apply_stiff(len(f), h, _d(f), _d(out))
    return out


def apply_advect(v, f):
    f = _f64(f)
    v = _f64(v)
    out = np.zeros_like(f)
    lib().orc_apply_advect(len(f), _d(v), _d(f), _d(out))
    return out


def velocity_from_momentum(model: Model, m):
    m = _f64(m)
    u = np.zeros_like(m)
    cm = model.c()
    st = lib().orc_velocity_from_momentum(C.byref(cm), _d(m), _d(u))
    assert st == ORC_OK, st
    return u


def momentum_from_velocity(model: Model, u):
    """m for each row of u (1-D or [particles][nx])."""
    u = _f64(u)
    cm = model.c()
    if u.ndim == 1:
        m = np.zeros_like(u)
        st = lib().orc_momentum_from_velocity(C.byref(cm), _d(u), _d(m))
        assert st == ORC_OK, st
        return m
    m = np.zeros_like(u)
    for p in range(u.shape[0]):
        row = np.ascontiguousarray(u[p])
        out = np.zeros_like(row)
        st = lib().orc_momentum_from_velocity(C.byref(cm), _d(row), _d(out))
        assert st == ORC_OK, st
        m[p] = out
    return m


def step(model: Model, m, u, dW, dLam=None):
    m = np.array(m, dtype=np.float64, copy=True)
    u = np.array(u, dtype=np.float64, copy=True)
    it = C.c_int32(0)
    cm = model.c()
    st = lib().orc_step(C.byref(cm), _d(m), _d(u), _d(_f64(dW)),
                        _d(_f64(dLam)) if dLam is not None else None, C.byref(it))
    return st, m, u, it.value


def window(model: Model, m, u, dW, dLam=None):
    m = np.array(m, dtype=np.float64, copy=True)
    u = np.array(u, dtype=np.float64, copy=True)
    dW = _f64(dW)
    it = C.c_int32(0)
    cm = model.c()
    st = lib().orc_window(C.byref(cm), dW.shape[0], _d(m), _d(u), _d(dW),
                          _d(_f64(dLam)) if dLam is not None else None, C.byref(it))
    return st, m, u, it.value


def ensemble_window(model: Model, m, u, dW, dLam=None, n_threads=None):
    """m, u: [P][nx]; dW: [P][n_steps][n_modes]. Returns (worst, m, u, status, iters)."""
    m = np.array(m, dtype=np.float64, copy=True, order="C")
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    dW = _f64(dW)
    P, ns = dW.shape[0], dW.shape[1]
    status = np.zeros(P, dtype=np.int32)
    iters = np.zeros(P, dtype=np.int32)
    cm = model.c()
    worst = lib().orc_ensemble_window(C.byref(cm), P, ns, _d(m), _d(u), _d(dW),
                                      _d(_f64(dLam)) if dLam is not None else None,
                                      _i(status), _i(iters), n_threads or n_threads_default())
    return worst, m, u, status, iters


# --------------------------------------------------------------------------- observation
def observe(u, n_obs):
    u = _f64(u)
    out = np.zeros(n_obs)
    lib().orc_observe(len(u), n_obs, _d(u), _d(out))
    return out


def nll(u, y, sigma):
    u = _f64(u)
    y = _f64(y)
    sigma = _f64(np.broadcast_to(sigma, y.shape))
    return lib().orc_nll(len(u), len(y), _d(u), _d(y), _d(sigma))


def ensemble_nll(u, y, sigma):
    u = _f64(u)
    y = _f64(y)
    sigma = _f64(np.broadcast_to(sigma, y.shape))
    phi = np.zeros(u.shape[0])
    lib().orc_ensemble_nll(u.shape[1], len(y), u.shape[0], _d(u), _d(y), _d(sigma), _d(phi))
    return phi


# --------------------------------------------------------------------------- weights
def weights(phi, beta, logw_extra=None):
    phi = _f64(phi)
    w = np.zeros_like(phi)
    lo = np.zeros_like(phi)
    ess = lib().orc_weights(len(phi), _d(phi), _d(_f64(logw_extra)) if logw_extra is not None
                            else None, beta, _d(w), _d(lo))
    return ess, w, lo


def temper(phi, theta, threshold, n_bisect=50):
    phi = _f64(phi)
    w = np.zeros_like(phi)
    dth = C.c_double(0)
    ess = C.c_double(0)
    lib().orc_temper(len(phi), _d(phi), theta, threshold, n_bisect, C.byref(dth), _d(w),
                     C.byref(ess))
    return dth.value, w, ess.value


def resample_systematic(w, u0):
    w = _f64(w)
    idx = np.zeros(len(w), dtype=np.int32)
    st = lib().orc_resample_systematic(len(w), _d(w), u0, _i(idx))
    return st, idx


def resample_textbook(w, u0):
    w = _f64(w)
    idx = np.zeros(len(w), dtype=np.int32)
    st = lib().orc_resample_textbook(len(w), _d(w), u0, _i(idx))
    return st, idx


# --------------------------------------------------------------------------- pCN
def jitter_pcn(model: Model, y, sigma, seed, cycle, temper_k, m0, u0, dW, phi, m_end, u_end,
               theta, rho, n_jitter, n_threads=None):
    y = _f64(y)
    sigma = _f64(np.broadcast_to(sigma, y.shape))
    dW = np.array(dW, dtype=np.float64, copy=True, order="C")
    phi = np.array(phi, dtype=np.float64, copy=True)
    m_end = np.array(m_end, dtype=np.float64, copy=True, order="C")
    u_end = np.array(u_end, dtype=np.float64, copy=True, order="C")
    P, ns = dW.shape[0], dW.shape[1]
    acc = np.zeros(P, dtype=np.int32)
    rg = OrcRng(seed, cycle, temper_k)
    cm = model.c()
    lib().orc_jitter_pcn(C.byref(cm), len(y), _d(y), _d(sigma), C.byref(rg), P, ns,
                         _d(_f64(m0)), _d(_f64(u0)), _d(dW), _d(phi), _d(m_end), _d(u_end),
                         theta, rho, n_jitter, _i(acc), n_threads or n_threads_default())
    return dW, phi, m_end, u_end, acc


def pcn_accept(theta, phi_old, phi_new, v) -> bool:
    return bool(lib().orc_pcn_accept(theta, phi_old, phi_new, v))


def pcn_linear_chain(seed, n_steps, n_modes, G, y, sigma, theta, rho, dt, n_iter, x0=None):
    G = _f64(G)
    y = _f64(y)
    d = n_steps * n_modes
    x0 = np.zeros(d) if x0 is None else _f64(x0)
    samples = np.zeros((n_iter, d))
    acc = lib().orc_pcn_linear_chain(seed, n_steps, n_modes, len(y), _d(G), _d(y), sigma, theta,
                                     rho, dt, n_iter, _d(x0), _d(samples))
    return samples, acc


# --------------------------------------------------------------------------- cycles
def bootstrap_cycle(model: Model, y, sigma, seed, cycle, m, u, logw, n_steps, ess_frac=0.5,
                    n_threads=None):
    """One bootstrap cycle, in place on copies; returns (rc, m, u, logw, stats)."""
    y = _f64(y)
    sigma = _f64(np.broadcast_to(sigma, y.shape))
    m = np.array(m, dtype=np.float64, copy=True, order="C")
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    logw = np.array(logw, dtype=np.float64, copy=True)
    st = OrcCycleStats()
    cm = model.c()
    rc = lib().orc_bootstrap_cycle(C.byref(cm), len(y), _d(y), _d(sigma), seed, cycle,
                                   m.shape[0], n_steps, ess_frac, _d(m), _d(u), _d(logw),
                                   C.byref(st), n_threads or n_threads_default())
    return rc, m, u, logw, st


def tempered_cycle(model: Model, y, sigma, seed, cycle, m, u, n_steps, ess_threshold,
                   n_bisect=50, rho=0.99, n_jitter=5, max_temper=100, n_threads=None):
    y = _f64(y)
    sigma = _f64(np.broadcast_to(sigma, y.shape))
    m = np.array(m, dtype=np.float64, copy=True, order="C")
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    st = OrcCycleStats()
    cm = model.c()
    rc = lib().orc_tempered_cycle(C.byref(cm), len(y), _d(y), _d(sigma), seed, cycle,
                                  m.shape[0], n_steps, ess_threshold, n_bisect, rho, n_jitter,
                                  max_temper, _d(m), _d(u), C.byref(st),
                                  n_threads or n_threads_default())
    return rc, m, u, st


PLANT_NONE = 0
PLANT_JITTER_PRE_THETA = 1
PLANT_CUMULATIVE_WEIGHTS = 2
PLANT_HMC_NO_KINETIC = 3


def tempered_cycle_linear(F, B, G, y, sigma, dt, seed, cycle, x, n_steps, n_modes,
                          ess_threshold, n_bisect=50, rho=0.99, n_jitter=5, max_temper=100,
                          plant=PLANT_NONE):
    """The tempering loop of the tempered drivers with the linear-Gaussian
    plug-in window e = F s + B xi, Phi = |G e - y|^2 / (2 sigma^2) (see
    orc_tempered_cycle_linear).  x [n][ds]: start states in; returns
    (rc, end states, stats)."""
    F, B, G, y = _f64(F), _f64(B), _f64(G), _f64(y)
    x = np.array(x, dtype=np.float64, copy=True, order="C")
    ds = x.shape[1]
    assert F.shape == (ds, ds) and B.shape == (ds, n_steps * n_modes) and G.shape == (len(y), ds)
    st = OrcCycleStats()
    rc = lib().orc_tempered_cycle_linear(ds, n_steps, n_modes, len(y), _d(F), _d(B), _d(G), _d(y),
                                         sigma, dt, seed, cycle, x.shape[0], ess_threshold,
                                         n_bisect, rho, n_jitter, max_temper, _d(x), C.byref(st),
                                         plant)
    return rc, x, st


# --------------------------------------------------------------------------- nudging
# L-BFGS settings of the nudging stages: memory 8, at most 30 accepted steps,
# stop at |grad|_inf <= 1e-8 (1 + |J|), at most 30 halvings per line search.
LBFGS_GTOL = 1e-8
LBFGS_MAX_ITER = 30
LBFGS_MEM = 8
LBFGS_MAX_BACK = 30


def _obs_arrays(y, sigma):
    y = _f64(y)
    return y, _f64(np.broadcast_to(sigma, y.shape))


def nudge_objective(model: Model, y, sigma, m0, u0, dW, dLam=None):
    """J = Phi(u^N) + sum_n (|dLam^n|^2/2 + dLam^n.dW^n)/dt (orc_nudge_objective)."""
    y, sg = _obs_arrays(y, sigma)
    dW = _f64(dW)
    J = C.c_double(0.0)
    cm = model.c()
    st = lib().orc_nudge_objective(C.byref(cm), len(y), _d(y), _d(sg), dW.shape[0],
                                   _d(_f64(m0)), _d(_f64(u0)), _d(dW),
                                   _d(_f64(dLam)) if dLam is not None else None, C.byref(J))
    return st, J.value


def nudge_grad(model: Model, y, sigma, m0, u0, dW, dLam=None):
    """Reverse-sweep adjoint: returns (status, J, dJ/ddLam [n_steps][Q]) (orc_nudge_grad)."""
    y, sg = _obs_arrays(y, sigma)
    dW = _f64(dW)
    J = C.c_double(0.0)
    g = np.zeros_like(dW)
    cm = model.c()
    st = lib().orc_nudge_grad(C.byref(cm), len(y), _d(y), _d(sg), dW.shape[0], _d(_f64(m0)),
                              _d(_f64(u0)), _d(dW),
                              _d(_f64(dLam)) if dLam is not None else None, C.byref(J), _d(g))
    return st, J.value, g


def nudge_grad_tangent(model: Model, y, sigma, m0, u0, dW, dLam=None):
    """Dense forward-mode gradient (small nx only) (orc_nudge_grad_tangent)."""
    y, sg = _obs_arrays(y, sigma)
    dW = _f64(dW)
    g = np.zeros_like(dW)
    cm = model.c()
    st = lib().orc_nudge_grad_tangent(C.byref(cm), len(y), _d(y), _d(sg), dW.shape[0],
                                      _d(_f64(m0)), _d(_f64(u0)), _d(dW),
                                      _d(_f64(dLam)) if dLam is not None else None, _d(g))
    return st, g


def lbfgs(fun, x0, h0=1.0, gtol=LBFGS_GTOL, max_iter=LBFGS_MAX_ITER, mem=LBFGS_MEM,
          max_back=LBFGS_MAX_BACK):
    """Run the oracle's L-BFGS on a Python objective fun(x) -> (status, f, g).
    Returns (status, x, f, iterations, evaluations)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    n = len(x)

    def cb(_ctx, xp, fp, gp):
        xv = np.ctypeslib.as_array(xp, shape=(n,)).copy()
        st, f, g = fun(xv)
        fp[0] = f
        for i in range(n):
            gp[i] = g[i]
        return int(st)

    cfun = OBJECTIVE(cb)
    f = C.c_double(0.0)
    it = C.c_int32(0)
    ev = C.c_int32(0)
    st = lib().orc_lbfgs(n, cfun, None, _d(x), h0, gtol, max_iter, mem, max_back, C.byref(f),
                         C.byref(it), C.byref(ev))
    return st, x, f.value, it.value, ev.value


def nudge_ensemble(model: Model, y, sigma, m, u, dW, dLam0=None, gtol=LBFGS_GTOL,
                   max_iter=LBFGS_MAX_ITER, mem=LBFGS_MEM, max_back=LBFGS_MAX_BACK,
                   n_threads=None):
    """Sequential adapted nudging of every particle over one window.
    m, u: [P][nx] (start state); dW: [P][S][Q] revealed increments; dLam0: warm
    start or None.  Returns dict(worst, m, u, dLam, logG, iters, evals,
    lbfgs_status, status)."""
    y, sg = _obs_arrays(y, sigma)
    m = np.array(m, dtype=np.float64, copy=True, order="C")
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    dW = _f64(dW)
    P, S = dW.shape[0], dW.shape[1]
    dLam = (np.zeros_like(dW) if dLam0 is None
            else np.array(dLam0, dtype=np.float64, copy=True, order="C"))
    logG = np.zeros(P)
    iters = np.zeros(P, dtype=np.int32)
    evals = np.zeros(P, dtype=np.int32)
    lst = np.zeros(P, dtype=np.int32)
    status = np.zeros(P, dtype=np.int32)
    opts = OrcLbfgsOpts(gtol, max_iter, mem, max_back)
    cm = model.c()
    worst = lib().orc_nudge_ensemble(C.byref(cm), len(y), _d(y), _d(sg), P, S, _d(m), _d(u),
                                     _d(dW), _d(dLam), C.byref(opts), _d(logG), _i(iters),
                                     _i(evals), _i(lst), _i(status),
                                     n_threads or n_threads_default())
    return dict(worst=worst, m=m, u=u, dLam=dLam, logG=logG, iters=iters, evals=evals,
                lbfgs_status=lst, status=status)


# --------------------------------------------------------------------------- nudged filter
def nudged_potential(phi, dt, dW, dLam) -> float:
    """phi - log G of one nudged path (flattened increments and controls)."""
    dW = _f64(np.ravel(dW))
    dLam = _f64(np.ravel(dLam))
    return lib().orc_nudged_potential(float(phi), len(dW), dt, _d(dW), _d(dLam))


def jitter_pcn_ctrl(model: Model, y, sigma, seed, cycle, temper_k, m0, u0, dW, dLam, J, m_end,
                    u_end, theta, rho, n_jitter, n_threads=None):
    """pCN moves of dW with the controls dLam fixed; J holds the nudged
    potentials.  Returns (dW, J, m_end, u_end, n_accept)."""
    y, sg = _obs_arrays(y, sigma)
    dW = np.array(dW, dtype=np.float64, copy=True, order="C")
    J = np.array(J, dtype=np.float64, copy=True)
    m_end = np.array(m_end, dtype=np.float64, copy=True, order="C")
    u_end = np.array(u_end, dtype=np.float64, copy=True, order="C")
    P, ns = dW.shape[0], dW.shape[1]
    acc = np.zeros(P, dtype=np.int32)
    rg = OrcRng(seed, cycle, temper_k)
    cm = model.c()
    lib().orc_jitter_pcn_ctrl(C.byref(cm), len(y), _d(y), _d(sg), C.byref(rg), P, ns,
                              _d(_f64(m0)), _d(_f64(u0)), _d(dW), _d(_f64(dLam)), _d(J),
                              _d(m_end), _d(u_end), theta, rho, n_jitter, _i(acc),
                              n_threads or n_threads_default())
    return dW, J, m_end, u_end, acc


def pcn_linear_chain_ctrl(seed, n_steps, n_modes, G, y, sigma, theta, rho, dt, lam, n_iter,
                          x0=None):
    G = _f64(G)
    y = _f64(y)
    d = n_steps * n_modes
    lam = _f64(np.ravel(lam))
    x0 = np.zeros(d) if x0 is None else _f64(x0)
    samples = np.zeros((n_iter, d))
    acc = lib().orc_pcn_linear_chain_ctrl(seed, n_steps, n_modes, len(y), _d(G), _d(y), sigma,
                                          theta, rho, dt, _d(lam), n_iter, _d(x0), _d(samples))
    return samples, acc


def nudged_cycle(model: Model, y, sigma, seed, cycle, m, u, n_steps, ess_threshold, n_bisect=50,
                 rho=0.99, n_jitter=5, max_temper=100, gtol=LBFGS_GTOL, max_iter=LBFGS_MAX_ITER,
                 mem=LBFGS_MEM, max_back=LBFGS_MAX_BACK, n_threads=None):
    """One cycle of the nudged filter (nudging, then tempering and jittering
    with the weights W~).  Returns (rc, out, stats) with out a dict of the
    window-end states m, u, the final window-start states m0, u0, increments
    dW, controls dLam and potentials J."""
    y, sg = _obs_arrays(y, sigma)
    m = np.array(m, dtype=np.float64, copy=True, order="C")
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    P = m.shape[0]
    m0 = np.zeros_like(m)
    u0 = np.zeros_like(u)
    dW = np.zeros((P, n_steps, model.n_modes))
    dLam = np.zeros_like(dW)
    J = np.zeros(P)
    st = OrcCycleStats()
    opts = OrcLbfgsOpts(gtol, max_iter, mem, max_back)
    cm = model.c()
    rc = lib().orc_nudged_cycle(C.byref(cm), len(y), _d(y), _d(sg), seed, cycle, P, n_steps,
                                ess_threshold, n_bisect, rho, n_jitter, max_temper,
                                C.byref(opts), _d(m), _d(u), _d(m0), _d(u0), _d(dW), _d(dLam),
                                _d(J), C.byref(st), n_threads or n_threads_default())
    return rc, dict(m=m, u=u, m0=m0, u0=u0, dW=dW, dLam=dLam, J=J), st


NUDGE_KEEP, NUDGE_FROM_GIVEN, NUDGE_FROM_ZERO = 0, 1, 2


def nudged_cycle_warm(model: Model, y, sigma, seed, cycle, m, u, dLam_start, mode, n_steps,
                      ess_threshold, n_bisect=50, rho=0.99, n_jitter=5, max_temper=100,
                      gtol=LBFGS_GTOL, max_iter=LBFGS_MAX_ITER, mem=LBFGS_MEM,
                      max_back=LBFGS_MAX_BACK, n_threads=None):
    """nudged_cycle with given start controls dLam_start [n][n_steps][Q] and a
    per-particle start mode (NUDGE_KEEP / NUDGE_FROM_GIVEN / NUDGE_FROM_ZERO)."""
    y, sg = _obs_arrays(y, sigma)
    m = np.array(m, dtype=np.float64, copy=True, order="C")
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    P = m.shape[0]
    lam0 = _f64(dLam_start)
    mode = np.ascontiguousarray(mode, dtype=np.int32)
    assert lam0.shape == (P, n_steps, model.n_modes) and mode.shape == (P,)
    m0, u0 = np.zeros_like(m), np.zeros_like(u)
    dW = np.zeros((P, n_steps, model.n_modes))
    dLam = np.zeros_like(dW)
    J = np.zeros(P)
    st = OrcCycleStats()
    opts = OrcLbfgsOpts(gtol, max_iter, mem, max_back)
    cm = model.c()
    rc = lib().orc_nudged_cycle_warm(C.byref(cm), len(y), _d(y), _d(sg), seed, cycle, P, n_steps,
                                     ess_threshold, n_bisect, rho, n_jitter, max_temper,
                                     C.byref(opts), _d(lam0), _i(mode), _d(m), _d(u), _d(m0),
                                     _d(u0), _d(dW), _d(dLam), _d(J), C.byref(st),
                                     n_threads or n_threads_default())
    return rc, dict(m=m, u=u, m0=m0, u0=u0, dW=dW, dLam=dLam, J=J), st


# --------------------------------------------------------------------------- Matern noise
def matern(kappa=1.0, eta=1.0, k=3) -> OrcMatern:
    return OrcMatern(kappa, eta, k)


def matern_field(nx, L, mt: OrcMatern, dWc):
    """Nodal Delta U of the Matern-type noise from the cell increments dWc [nx]."""
    dWc = _f64(dWc)
    out = np.zeros(nx)
    st = lib().orc_matern_field(nx, L, C.byref(mt), _d(dWc), _d(out))
    assert st == ORC_OK, st
    return out


def step_field(model: Model, m, u, dU):
    m = np.array(m, dtype=np.float64, copy=True)
    u = np.array(u, dtype=np.float64, copy=True)
    it = C.c_int32(0)
    cm = model.c()
    st = lib().orc_step_field(C.byref(cm), _d(m), _d(u), _d(_f64(dU)), C.byref(it))
    return st, m, u, it.value


def window_matern(model: Model, mt: OrcMatern, m, u, dWc):
    m = np.array(m, dtype=np.float64, copy=True)
    u = np.array(u, dtype=np.float64, copy=True)
    dWc = _f64(dWc)
    it = C.c_int32(0)
    cm = model.c()
    st = lib().orc_window_matern(C.byref(cm), C.byref(mt), dWc.shape[0], _d(m), _d(u), _d(dWc),
                                 C.byref(it))
    return st, m, u, it.value


def ensemble_window_matern(model: Model, mt: OrcMatern, m, u, dWc, n_threads=None):
    m = np.array(m, dtype=np.float64, copy=True, order="C")
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    dWc = _f64(dWc)
    P, S = dWc.shape[0], dWc.shape[1]
    status = np.zeros(P, dtype=np.int32)
    iters = np.zeros(P, dtype=np.int32)
    cm = model.c()
    worst = lib().orc_ensemble_window_matern(C.byref(cm), C.byref(mt), P, S, _d(m), _d(u),
                                             _d(dWc), _i(status), _i(iters),
                                             n_threads or n_threads_default())
    return worst, m, u, status, iters


def jitter_pcn_matern(model: Model, mt: OrcMatern, y, sigma, seed, cycle, temper_k, m0, u0, dWc,
                      phi, m_end, u_end, theta, rho, n_jitter, n_threads=None):
    y, sg = _obs_arrays(y, sigma)
    dWc = np.array(dWc, dtype=np.float64, copy=True, order="C")
    phi = np.array(phi, dtype=np.float64, copy=True)
    m_end = np.array(m_end, dtype=np.float64, copy=True, order="C")
    u_end = np.array(u_end, dtype=np.float64, copy=True, order="C")
    P, ns = dWc.shape[0], dWc.shape[1]
    acc = np.zeros(P, dtype=np.int32)
    rg = OrcRng(seed, cycle, temper_k)
    cm = model.c()
    lib().orc_jitter_pcn_matern(C.byref(cm), C.byref(mt), len(y), _d(y), _d(sg), C.byref(rg), P,
                                ns, _d(_f64(m0)), _d(_f64(u0)), _d(dWc), _d(phi), _d(m_end),
                                _d(u_end), theta, rho, n_jitter, _i(acc),
                                n_threads or n_threads_default())
    return dWc, phi, m_end, u_end, acc


def bootstrap_cycle_matern(model: Model, mt: OrcMatern, y, sigma, seed, cycle, m, u, logw,
                           n_steps, ess_frac=0.5, n_threads=None):
    """bootstrap_cycle with the Matern-type noise; returns (rc, m, u, logw, stats)."""
    y, sg = _obs_arrays(y, sigma)
    m = np.array(m, dtype=np.float64, copy=True, order="C")
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    logw = np.array(logw, dtype=np.float64, copy=True)
    st = OrcCycleStats()
    cm = model.c()
    rc = lib().orc_bootstrap_cycle_matern(C.byref(cm), C.byref(mt), len(y), _d(y), _d(sg), seed,
                                          cycle, m.shape[0], n_steps, ess_frac, _d(m), _d(u),
                                          _d(logw), C.byref(st), n_threads or n_threads_default())
    return rc, m, u, logw, st


def tempered_cycle_matern(model: Model, mt: OrcMatern, y, sigma, seed, cycle, m, u, n_steps,
                          ess_threshold, n_bisect=50, rho=0.99, n_jitter=5, max_temper=100,
                          n_threads=None):
    """Tempered + jittered cycle with the Matern-type noise.  Returns (rc, out,
    stats), out holding m, u (window ends), m0, u0, dWc, phi."""
    y, sg = _obs_arrays(y, sigma)
    m = np.array(m, dtype=np.float64, copy=True, order="C")
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    P, nx = m.shape
    m0, u0 = np.zeros_like(m), np.zeros_like(u)
    dWc = np.zeros((P, n_steps, nx))
    phi = np.zeros(P)
    st = OrcCycleStats()
    cm = model.c()
    rc = lib().orc_tempered_cycle_matern(C.byref(cm), C.byref(mt), len(y), _d(y), _d(sg), seed,
                                         cycle, P, n_steps, ess_threshold, n_bisect, rho,
                                         n_jitter, max_temper, _d(m), _d(u), _d(m0), _d(u0),
                                         _d(dWc), _d(phi), C.byref(st),
                                         n_threads or n_threads_default())
    return rc, dict(m=m, u=u, m0=m0, u0=u0, dWc=dWc, phi=phi), st


# --------------------------------------------------------------------------- section 4
def paper_init_from(nx, L, W, alpha, beta):
    """Initial velocity of eq. init_solve from the cell values W [nx] and alpha, beta."""
    u = np.zeros(nx)
    st = lib().orc_paper_init_from(nx, L, _d(_f64(W)), alpha, beta, _d(u))
    assert st == ORC_OK, st
    return u


def paper_init(nx, L, seed, n, p0=0):
    """Rows p0 .. p0 + n - 1 of the paper's initial ensemble (Philox tag INIT)."""
    u = np.zeros((n, nx))
    st = lib().orc_paper_init(nx, L, seed, p0, n, _d(u))
    assert st == ORC_OK, st
    return u


def ensemble_stats(u, ua):
    """(EMRE, RB, RES) of the ensemble u [n][nx] against the truth ua [nx]."""
    u = _f64(np.atleast_2d(u))
    out = np.zeros(3)
    lib().orc_ensemble_stats(u.shape[0], u.shape[1], _d(u), _d(_f64(ua)), _d(out))
    return out


# --------------------------------------------------------------------------- pCN Langevin
def pcnl_log_ratio(x, phi_x, g_x, v, phi_v, g_v, theta, rho, dt) -> float:
    x, g_x, v, g_v = (_f64(a) for a in (x, g_x, v, g_v))
    return lib().orc_pcnl_log_ratio(len(x), _d(x), phi_x, _d(g_x), _d(v), phi_v, _d(g_v), theta,
                                    rho, dt)


def pcnl_linear_chain(seed, n_steps, n_modes, G, y, sigma, theta, rho, dt, n_iter, x0=None):
    G = _f64(G)
    y = _f64(y)
    d = n_steps * n_modes
    x0 = np.zeros(d) if x0 is None else _f64(x0)
    samples = np.zeros((n_iter, d))
    acc = lib().orc_pcnl_linear_chain(seed, n_steps, n_modes, len(y), _d(G), _d(y), sigma, theta,
                                      rho, dt, n_iter, _d(x0), _d(samples))
    return samples, acc


def jitter_pcnl(model: Model, y, sigma, seed, cycle, temper_k, m0, u0, dW, phi, theta, rho,
                n_jitter, n_threads=None):
    """pCN-Langevin moves; returns (dW, phi, m_end, u_end, n_accept)."""
    y, sg = _obs_arrays(y, sigma)
    dW = np.array(dW, dtype=np.float64, copy=True, order="C")
    phi = np.array(phi, dtype=np.float64, copy=True)
    P, ns = dW.shape[0], dW.shape[1]
    m_end = np.zeros((P, model.nx))
    u_end = np.zeros((P, model.nx))
    acc = np.zeros(P, dtype=np.int32)
    rg = OrcRng(seed, cycle, temper_k)
    cm = model.c()
    lib().orc_jitter_pcnl(C.byref(cm), len(y), _d(y), _d(sg), C.byref(rg), P, ns, _d(_f64(m0)),
                          _d(_f64(u0)), _d(dW), _d(phi), _d(m_end), _d(u_end), theta, rho,
                          n_jitter, _i(acc), n_threads or n_threads_default())
    return dW, phi, m_end, u_end, acc


def tempered_cycle_pcnl(model: Model, y, sigma, seed, cycle, m, u, n_steps, ess_threshold,
                        n_bisect=50, rho=0.99, n_jitter=5, max_temper=100, n_threads=None):
    y, sg = _obs_arrays(y, sigma)
    m = np.array(m, dtype=np.float64, copy=True, order="C")
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    st = OrcCycleStats()
    cm = model.c()
    rc = lib().orc_tempered_cycle_pcnl(C.byref(cm), len(y), _d(y), _d(sg), seed, cycle,
                                       m.shape[0], n_steps, ess_threshold, n_bisect, rho,
                                       n_jitter, max_temper, _d(m), _d(u), C.byref(st),
                                       n_threads or n_threads_default())
    return rc, m, u, st


# --------------------------------------------------------------------------- Hybrid Monte Carlo
def hmc_trajectory_linear(G, y, sigma, theta, h, n_leap, dt, x, v):
    """n_leap leapfrog steps of the HMC integrator for the linear-Gaussian toy
    Phi(x) = |G x - y|^2 / (2 sigma^2); returns the final (x, v)."""
    G = _f64(G)
    y = _f64(y)
    x = np.array(x, dtype=np.float64, copy=True)
    v = np.array(v, dtype=np.float64, copy=True)
    lib().orc_hmc_trajectory_linear(len(x), len(y), _d(G), _d(y), sigma, theta, h, n_leap, dt,
                                    _d(x), _d(v))
    return x, v


def hmc_linear_chain(seed, n_steps, n_modes, G, y, sigma, theta, h, n_leap, dt, n_iter,
                     x0=None, plant=0):
    G = _f64(G)
    y = _f64(y)
    d = n_steps * n_modes
    x0 = np.zeros(d) if x0 is None else _f64(x0)
    samples = np.zeros((n_iter, d))
    acc = lib().orc_hmc_linear_chain(seed, n_steps, n_modes, len(y), _d(G), _d(y), sigma, theta,
                                     h, n_leap, dt, n_iter, _d(x0), _d(samples), plant)
    return samples, acc


def jitter_hmc(model: Model, y, sigma, seed, cycle, temper_k, m0, u0, dW, phi, theta, h, n_leap,
               n_jitter, n_threads=None):
    """Hybrid Monte Carlo moves; returns (rc, dW, phi, m_end, u_end, n_accept)."""
    y, sg = _obs_arrays(y, sigma)
    dW = np.array(dW, dtype=np.float64, copy=True, order="C")
    phi = np.array(phi, dtype=np.float64, copy=True)
    P, ns = dW.shape[0], dW.shape[1]
    m_end = np.zeros((P, model.nx))
    u_end = np.zeros((P, model.nx))
    acc = np.zeros(P, dtype=np.int32)
    rg = OrcRng(seed, cycle, temper_k)
    cm = model.c()
    rc = lib().orc_jitter_hmc(C.byref(cm), len(y), _d(y), _d(sg), C.byref(rg), P, ns,
                              _d(_f64(m0)), _d(_f64(u0)), _d(dW), _d(phi), _d(m_end), _d(u_end),
                              theta, h, n_leap, n_jitter, _i(acc), n_threads or n_threads_default())
    return rc, dW, phi, m_end, u_end, acc


def tempered_cycle_hmc(model: Model, y, sigma, seed, cycle, m, u, n_steps, ess_threshold,
                       n_bisect=50, h=0.3, n_leap=3, n_jitter=5, max_temper=100, n_threads=None):
    y, sg = _obs_arrays(y, sigma)
    m = np.array(m, dtype=np.float64, copy=True, order="C")
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    st = OrcCycleStats()
    cm = model.c()
    rc = lib().orc_tempered_cycle_hmc(C.byref(cm), len(y), _d(y), _d(sg), seed, cycle,
                                      m.shape[0], n_steps, ess_threshold, n_bisect, h, n_leap,
                                      n_jitter, max_temper, _d(m), _d(u), C.byref(st),
                                      n_threads or n_threads_default())
    return rc, m, u, st


# --------------------------------------------------------------------------- Matern nudging
def matern_transpose(nx, L, mt: OrcMatern, g):
    """The transpose of matern_field's linear map, applied to g [nx]."""
    out = np.zeros(nx)
    st = lib().orc_matern_transpose(nx, L, C.byref(mt), _d(_f64(g)), _d(out))
    assert st == ORC_OK, st
    return out


def nudge_grad_matern(model: Model, mt: OrcMatern, y, sigma, m0, u0, dW, dLam=None):
    """(status, J, dJ/ddLam [n_steps][nx]) with the Matern-type noise."""
    y, sg = _obs_arrays(y, sigma)
    dW = _f64(dW)
    J = C.c_double(0.0)
    g = np.zeros_like(dW)
    cm = model.c()
    st = lib().orc_nudge_grad_matern(C.byref(cm), C.byref(mt), len(y), _d(y), _d(sg),
                                     dW.shape[0], _d(_f64(m0)), _d(_f64(u0)), _d(dW),
                                     _d(_f64(dLam)) if dLam is not None else None, C.byref(J),
                                     _d(g))
    return st, J.value, g


def nudge_ensemble_matern(model: Model, mt: OrcMatern, y, sigma, m, u, dW, dLam0=None,
                          gtol=LBFGS_GTOL, max_iter=LBFGS_MAX_ITER, mem=LBFGS_MEM,
                          max_back=LBFGS_MAX_BACK, n_threads=None):
    """nudge_ensemble with the Matern-type noise (controls per cell)."""
    y, sg = _obs_arrays(y, sigma)
    m = np.array(m, dtype=np.float64, copy=True, order="C")
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    dW = _f64(dW)
    P, S = dW.shape[0], dW.shape[1]
    dLam = (np.zeros_like(dW) if dLam0 is None
            else np.array(dLam0, dtype=np.float64, copy=True, order="C"))
    logG = np.zeros(P)
    iters = np.zeros(P, dtype=np.int32)
    evals = np.zeros(P, dtype=np.int32)
    lst = np.zeros(P, dtype=np.int32)
    status = np.zeros(P, dtype=np.int32)
    opts = OrcLbfgsOpts(gtol, max_iter, mem, max_back)
    cm = model.c()
    worst = lib().orc_nudge_ensemble_matern(C.byref(cm), C.byref(mt), len(y), _d(y), _d(sg), P,
                                            S, _d(m), _d(u), _d(dW), _d(dLam), C.byref(opts),
                                            _d(logG), _i(iters), _i(evals), _i(lst), _i(status),
                                            n_threads or n_threads_default())
    return dict(worst=worst, m=m, u=u, dLam=dLam, logG=logG, iters=iters, evals=evals,
                lbfgs_status=lst, status=status)


def jitter_pcn_matern_ctrl(model: Model, mt: OrcMatern, y, sigma, seed, cycle, temper_k, m0, u0,
                           dWc, dLamc, J, m_end, u_end, theta, rho, n_jitter, n_threads=None):
    """pCN moves of the cells dWc with the per-cell controls dLamc fixed; J
    holds the nudged potentials.  Returns (dWc, J, m_end, u_end, n_accept)."""
    y, sg = _obs_arrays(y, sigma)
    dWc = np.array(dWc, dtype=np.float64, copy=True, order="C")
    J = np.array(J, dtype=np.float64, copy=True)
    m_end = np.array(m_end, dtype=np.float64, copy=True, order="C")
    u_end = np.array(u_end, dtype=np.float64, copy=True, order="C")
    P, ns = dWc.shape[0], dWc.shape[1]
    acc = np.zeros(P, dtype=np.int32)
    rg = OrcRng(seed, cycle, temper_k)
    cm = model.c()
    lib().orc_jitter_pcn_matern_ctrl(C.byref(cm), C.byref(mt), len(y), _d(y), _d(sg),
                                     C.byref(rg), P, ns, _d(_f64(m0)), _d(_f64(u0)), _d(dWc),
                                     _d(_f64(dLamc)), _d(J), _d(m_end), _d(u_end), theta, rho,
                                     n_jitter, _i(acc), n_threads or n_threads_default())
    return dWc, J, m_end, u_end, acc


def nudged_cycle_matern(model: Model, mt: OrcMatern, y, sigma, seed, cycle, m, u, n_steps,
                        ess_threshold, n_bisect=50, rho=0.99, n_jitter=5, max_temper=100,
                        gtol=LBFGS_GTOL, max_iter=LBFGS_MAX_ITER, mem=LBFGS_MEM,
                        max_back=LBFGS_MAX_BACK, n_threads=None):
    """nudged_cycle with the Matern-type noise (increments and controls per
    cell); returns (rc, out, stats) as nudged_cycle."""
    y, sg = _obs_arrays(y, sigma)
    m = np.array(m, dtype=np.float64, copy=True, order="C")
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    P, nx = m.shape
    m0 = np.zeros_like(m)
    u0 = np.zeros_like(u)
    dW = np.zeros((P, n_steps, nx))
    dLam = np.zeros_like(dW)
    J = np.zeros(P)
    st = OrcCycleStats()
    opts = OrcLbfgsOpts(gtol, max_iter, mem, max_back)
    cm = model.c()
    rc = lib().orc_nudged_cycle_matern(C.byref(cm), C.byref(mt), len(y), _d(y), _d(sg), seed,
                                       cycle, P, n_steps, ess_threshold, n_bisect, rho, n_jitter,
                                       max_temper, C.byref(opts), _d(m), _d(u), _d(m0), _d(u0),
                                       _d(dW), _d(dLam), _d(J), C.byref(st),
                                       n_threads or n_threads_default())
    return rc, dict(m=m, u=u, m0=m0, u0=u0, dW=dW, dLam=dLam, J=J), st
