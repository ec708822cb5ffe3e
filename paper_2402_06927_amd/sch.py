"""ctypes binding of the C-ABI in include/sch.h.

Argument marshalling only: every function takes torch tensors that live on
the GPU, checks dtype / contiguity / device, and passes raw device pointers
and the current HIP stream to ``libsch.so``.  All arithmetic of the method
runs in the library's kernels.  There is no fallback: if the library is not
built, or a tensor is not on the GPU, the call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsch.so")
_lib = None

SCH_OK = 0
SCH_E_ARG = -1
SCH_E_SHAPE = -2
SCH_E_NONCONVERGED = -3
SCH_E_NONFINITE = -4
SCH_E_DEGENERATE = -5
SCH_E_HIP = -6
SCH_E_UNSTABLE = -7

TAG_INIT, TAG_FORECAST, TAG_PCN, TAG_ACCEPT, TAG_RESAMPLE, TAG_OBS, TAG_NUDGE = range(7)
WS_RESAMPLE, WS_BOOTSTRAP, WS_TEMPERED, WS_JITTER, WS_NUDGE_GRAD, WS_NUDGE = 1, 2, 3, 4, 5, 6


class SchError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sch error {code}: {msg}")
        self.code = code


_vp = C.c_void_p


class SchModelC(C.Structure):
    _fields_ = [
        ("L", C.c_double), ("alpha", C.c_double), ("mu", C.c_double), ("dt", C.c_double),
        ("nx", C.c_int32), ("n_modes", C.c_int32), ("xi", _vp),
        ("picard_tol", C.c_double), ("picard_max", C.c_int32),
    ]


class SchObsC(C.Structure):
    _fields_ = [("n_obs", C.c_int32), ("y", _vp), ("sigma", _vp)]


class SchRngC(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("cycle", C.c_uint32), ("temper_k", C.c_uint32)]


class SchMaternC(C.Structure):
    _fields_ = [("kappa", C.c_double), ("eta", C.c_double), ("k", C.c_int32)]


class SchCycleStats(C.Structure):
    _fields_ = [
        ("ess", C.c_double), ("resampled", C.c_int32), ("n_temper", C.c_int32),
        ("picard_iters", C.c_int64), ("n_accept", C.c_int64), ("particle_steps", C.c_int64),
        ("status", C.c_int32), ("n_failed", C.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SchInstanceC(C.Structure):
    _fields_ = [("nx", C.c_int32), ("n_particles", C.c_int32), ("xi", _vp), ("m", _vp),
                ("u", _vp), ("logw", _vp), ("y", _vp), ("sigma", _vp), ("seed", C.c_uint64),
                ("threads", C.c_int32)]


class SchBatchParamsC(C.Structure):
    _fields_ = [("L", C.c_double), ("alpha", C.c_double), ("mu", C.c_double),
                ("dt", C.c_double), ("n_modes", C.c_int32), ("n_steps", C.c_int32),
                ("n_obs", C.c_int32), ("ess_frac", C.c_double), ("picard_tol", C.c_double),
                ("picard_max", C.c_int32)]


class SchMlpC(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_hidden", C.c_int32), ("n_out", C.c_int32),
                ("params", _vp), ("weights_bf16", _vp)]


class SchLbfgsOpts(C.Structure):
    _fields_ = [("gtol", C.c_double), ("max_iter", C.c_int32), ("mem", C.c_int32),
                ("max_back", C.c_int32)]


def lib():
    """Load libsch.so (built in place by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


def _declare(L):
    i32, u32, u64, i64, f64 = C.c_int32, C.c_uint32, C.c_uint64, C.c_int64, C.c_double
    M, O, R = C.POINTER(SchModelC), C.POINTER(SchObsC), C.POINTER(SchRngC)
    ST = C.POINTER(SchCycleStats)
    MT = C.POINTER(SchMaternC)
    sig = {
        "sch_last_error": (C.c_char_p, []),
        "sch_version": (C.c_int, []),
        "sch_workspace_bytes": (C.c_size_t, [i32, M, i32, i32, i32]),
        "sch_draw_increments": (C.c_int, [R, u32, i32, i32, i32, f64, _vp, _vp]),
        "sch_philox_blocks": (C.c_int, [u64, i32, _vp, _vp, _vp]),
        "sch_velocity": (C.c_int, [M, i32, _vp, _vp, _vp]),
        "sch_init_momentum": (C.c_int, [M, i32, _vp, _vp, _vp]),
        "sch_ensemble_step": (C.c_int, [M, i32, i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
        "sch_observe": (C.c_int, [M, i32, i32, _vp, _vp, _vp]),
        "sch_loglik": (C.c_int, [M, O, i32, _vp, _vp, _vp]),
        "sch_temper_ess": (C.c_int, [i32, _vp, _vp, _vp, f64, i32, _vp, _vp, _vp, _vp, _vp]),
        "sch_resample": (C.c_int, [i32, _vp, _vp, _vp, f64, _vp, _vp, _vp, _vp]),
        "sch_gather": (C.c_int, [i32, i64, _vp, _vp, _vp, _vp]),
        "sch_jitter_pcn": (C.c_int, [M, O, R, i32, i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                     _vp, f64, i32, _vp, _vp, _vp]),
        "sch_jitter_pcn_noalloc_max_bytes": (C.c_size_t, []),
        "sch_jitter_pcn_noalloc": (C.c_int, [M, O, R, i32, i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                             _vp, _vp, f64, i32, _vp, _vp]),
        "sch_pf_bootstrap_cycle": (C.c_int, [M, O, u64, u32, i32, i32, f64, _vp, _vp, _vp, _vp,
                                             ST, _vp]),
        "sch_pf_tempered_cycle": (C.c_int, [M, O, u64, u32, i32, i32, f64, i32, f64, i32, i32,
                                            _vp, _vp, _vp, ST, _vp]),
        "sch_nudged_workspace_bytes": (C.c_size_t, [M, i32, i32, i32, i32]),
        "sch_pf_nudged_cycle": (C.c_int, [M, O, u64, u32, i32, i32, f64, i32, f64, i32, i32,
                                          C.POINTER(SchLbfgsOpts), i32, _vp, _vp, _vp, _vp, ST,
                                          _vp]),
        "sch_pf_nudged_cycle_warm": (C.c_int, [M, O, u64, u32, i32, i32, f64, i32, f64, i32,
                                               i32, C.POINTER(SchLbfgsOpts), i32, _vp, _vp, _vp,
                                               _vp, _vp, ST, _vp]),
        "sch_nudge_grad": (C.c_int, [M, O, i32, i32, _vp, _vp, _vp, _vp, i32, _vp, _vp, _vp,
                                     _vp, _vp]),
        "sch_nudge_run": (C.c_int, [M, O, i32, i32, _vp, _vp, _vp, _vp, i32,
                                    C.POINTER(SchLbfgsOpts), i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                    _vp]),
        "sch_batch_workspace_bytes": (C.c_size_t, [C.POINTER(SchBatchParamsC), i32,
                                                   C.POINTER(SchInstanceC)]),
        "sch_batch_create": (C.c_int, [C.POINTER(SchBatchParamsC), i32, C.POINTER(SchInstanceC),
                                       _vp, C.c_size_t, C.POINTER(_vp), _vp]),
        "sch_batch_run": (C.c_int, [_vp, u32, i32, i32, _vp]),
        "sch_batch_read": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
        "sch_batch_destroy": (C.c_int, [_vp]),
        "sch_mlp_param_count": (C.c_size_t, [i32, i32, i32]),
        "sch_mlp_workspace_bytes": (C.c_size_t, [C.POINTER(SchMlpC), i32]),
        "sch_mlp_sync": (C.c_int, [C.POINTER(SchMlpC), _vp]),
        "sch_mlp_forward": (C.c_int, [C.POINTER(SchMlpC), i32, _vp, _vp, _vp, _vp]),
        "sch_mlp_backward": (C.c_int, [C.POINTER(SchMlpC), i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                       _vp]),
        "sch_mlp_adam": (C.c_int, [C.POINTER(SchMlpC), _vp, _vp, _vp, i32, C.c_float,
                                   C.c_float, C.c_float, C.c_float, _vp]),
        "sch_mlp_features": (C.c_int, [M, O, i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
        "sch_mlp_colstats": (C.c_int, [i32, i32, _vp, _vp, _vp, _vp]),
        "sch_mlp_encode": (C.c_int, [i32, i32, _vp, _vp, _vp, _vp, _vp]),
        "sch_mlp_targets": (C.c_int, [i32, i32, _vp, _vp, _vp, _vp, _vp]),
        "sch_mlp_controls": (C.c_int, [i32, i32, _vp, _vp, _vp, _vp, f64, _vp, _vp, i32, _vp]),
        "sch_tune_set": (C.c_int, [i32, i32]),
        "sch_tune_get": (C.c_int, [i32]),
        "sch_timing_enable": (C.c_int, [C.c_int]),
        "sch_timing_reset": (C.c_int, []),
        "sch_timing_read": (C.c_int, [C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64)]),
        "sch_matern_field": (C.c_int, [M, MT, i32, _vp, _vp, _vp]),
        "sch_ensemble_step_matern": (C.c_int, [M, MT, i32, i32, _vp, _vp, _vp, _vp, _vp, _vp]),
        "sch_matern_workspace_bytes": (C.c_size_t, [i32, M, i32, i32, i32]),
        "sch_jitter_pcn_matern": (C.c_int, [M, MT, O, R, i32, i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                            _vp, f64, i32, _vp, _vp, _vp]),
        "sch_pf_tempered_cycle_matern": (C.c_int, [M, MT, O, u64, u32, i32, i32, f64, i32, f64,
                                                   i32, i32, _vp, _vp, _vp, ST, _vp]),
        "sch_pf_bootstrap_cycle_matern": (C.c_int, [M, MT, O, u64, u32, i32, i32, f64, _vp, _vp,
                                                    _vp, _vp, ST, _vp]),
        "sch_paper_init": (C.c_int, [M, u64, i32, _vp, _vp]),
        "sch_pcnl_workspace_bytes": (C.c_size_t, [i32, M, i32, i32, i32, i32]),
        "sch_jitter_pcnl": (C.c_int, [M, O, R, i32, i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, f64,
                                      i32, i32, _vp, _vp, _vp]),
        "sch_pf_tempered_cycle_pcnl": (C.c_int, [M, O, u64, u32, i32, i32, f64, i32, f64, i32,
                                                 i32, i32, _vp, _vp, _vp, ST, _vp]),
        "sch_hmc_workspace_bytes": (C.c_size_t, [i32, M, i32, i32, i32, i32]),
        "sch_jitter_hmc": (C.c_int, [M, O, R, i32, i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, f64,
                                     i32, i32, i32, _vp, _vp, _vp]),
        "sch_pf_tempered_cycle_hmc": (C.c_int, [M, O, u64, u32, i32, i32, f64, i32, f64, i32, i32,
                                                i32, i32, _vp, _vp, _vp, ST, _vp]),
        "sch_ensemble_stats": (C.c_int, [i32, i32, _vp, _vp, _vp, _vp, _vp]),
        "sch_nudge_grad_matern": (C.c_int, [M, MT, O, i32, i32, _vp, _vp, _vp, _vp, i32, _vp,
                                            _vp, _vp, _vp, _vp]),
        "sch_nudge_run_matern": (C.c_int, [M, MT, O, i32, i32, _vp, _vp, _vp, _vp, i32,
                                           C.POINTER(SchLbfgsOpts), i32, _vp, _vp, _vp, _vp, _vp,
                                           _vp, _vp]),
        "sch_nudged_workspace_bytes_matern": (C.c_size_t, [M, i32, i32, i32, i32]),
        "sch_jitter_pcn_matern_ctrl": (C.c_int, [M, MT, O, R, i32, i32, _vp, _vp, _vp, _vp, _vp,
                                                 _vp, _vp, _vp, f64, i32, _vp, _vp, _vp]),
        "sch_pf_nudged_cycle_matern": (C.c_int, [M, MT, O, u64, u32, i32, i32, f64, i32, f64, i32,
                                                 i32, C.POINTER(SchLbfgsOpts), i32, _vp, _vp, _vp,
                                                 _vp, ST, _vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def exported_names():
    """Names of the C-ABI entry points this binding declares."""
    return [
        "sch_last_error", "sch_version", "sch_workspace_bytes", "sch_draw_increments",
        "sch_philox_blocks",
        "sch_velocity", "sch_init_momentum", "sch_ensemble_step", "sch_observe", "sch_loglik",
        "sch_temper_ess", "sch_resample", "sch_gather", "sch_jitter_pcn",
        "sch_jitter_pcn_noalloc_max_bytes", "sch_jitter_pcn_noalloc", "sch_nudge_grad", "sch_nudge_run", "sch_pf_bootstrap_cycle",
        "sch_batch_workspace_bytes", "sch_batch_create", "sch_batch_run", "sch_batch_read",
        "sch_batch_destroy", "sch_mlp_param_count", "sch_mlp_workspace_bytes", "sch_mlp_sync",
        "sch_mlp_forward", "sch_mlp_backward", "sch_mlp_adam", "sch_mlp_features",
        "sch_mlp_colstats", "sch_mlp_encode", "sch_mlp_targets", "sch_mlp_controls",
        "sch_pf_tempered_cycle", "sch_nudged_workspace_bytes", "sch_pf_nudged_cycle",
        "sch_pf_nudged_cycle_warm",
        "sch_tune_set", "sch_tune_get", "sch_timing_enable", "sch_timing_reset",
        "sch_timing_read", "sch_matern_field", "sch_ensemble_step_matern",
        "sch_matern_workspace_bytes", "sch_jitter_pcn_matern", "sch_pf_tempered_cycle_matern",
        "sch_pf_bootstrap_cycle_matern", "sch_paper_init", "sch_ensemble_stats",
        "sch_pcnl_workspace_bytes", "sch_jitter_pcnl", "sch_pf_tempered_cycle_pcnl",
        "sch_hmc_workspace_bytes", "sch_jitter_hmc", "sch_pf_tempered_cycle_hmc",
        "sch_nudge_grad_matern", "sch_nudge_run_matern", "sch_nudged_workspace_bytes_matern",
        "sch_pf_nudged_cycle_matern", "sch_jitter_pcn_matern_ctrl",
    ]


def _check(rc: int):
    if rc != SCH_OK:
        raise SchError(rc, lib().sch_last_error().decode())


def _dev(t: torch.Tensor | None, dtype=torch.float64, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _shape(t: torch.Tensor | None, shape: tuple, name: str):
    """Raise SchError(SCH_E_SHAPE) unless t (if given) has exactly `shape`;
    the kernels index the caller's arrays from these sizes, so a mismatch
    would read or write outside them on the device."""
    if t is None:
        return
    if tuple(t.shape) != tuple(int(d) for d in shape):
        raise SchError(SCH_E_SHAPE, f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _at_least(t: torch.Tensor | None, numel: int, name: str):
    if t is None:
        return
    if t.numel() < numel:
        raise SchError(SCH_E_SHAPE, f"{name} has {t.numel()} elements, needs at least {numel}")


def _ws(ws: torch.Tensor, nbytes: int, name: str = "workspace"):
    """The workspace must hold the bytes its *_workspace_bytes query gives."""
    if nbytes <= 0:
        raise SchError(SCH_E_ARG, f"invalid {name} request")
    have = ws.numel() * ws.element_size()
    if have < nbytes:
        raise SchError(SCH_E_SHAPE, f"{name} has {have} bytes, the call needs {nbytes}")


def _state(model: "Model", n: int, **arrays):
    for k, v in arrays.items():
        _shape(v, (n, model.nx), k)


def _inc(n: int, s: int, q: int, **arrays):
    for k, v in arrays.items():
        _shape(v, (n, s, q), k)


def _vec(n: int, **arrays):
    for k, v in arrays.items():
        _shape(v, (n,), k)


@dataclass
class Model:
    """SCH model parameters (section 2) with the noise-mode table on the GPU."""
    L: float
    alpha: float
    mu: float
    dt: float
    xi: torch.Tensor  # [n_modes][nx] float64 on the GPU
    picard_tol: float = 1e-13
    picard_max: int = 50

    @property
    def nx(self) -> int:
        return int(self.xi.shape[1])

    @property
    def n_modes(self) -> int:
        return int(self.xi.shape[0])

    def c(self) -> SchModelC:
        return SchModelC(self.L, self.alpha, self.mu, self.dt, self.nx, self.n_modes,
                         _dev(self.xi, name="xi"), self.picard_tol, self.picard_max)


@dataclass
class Obs:
    y: torch.Tensor      # [n_obs]
    sigma: torch.Tensor  # [n_obs]

    def c(self) -> SchObsC:
        _shape(self.sigma, tuple(self.y.shape), "sigma")
        return SchObsC(int(self.y.numel()), _dev(self.y, name="y"), _dev(self.sigma, name="sigma"))


def workspace_bytes(which: int, model: Model | None, n_particles: int, n_steps: int = 0,
                    extra: int = 0) -> int:
    """Bytes of scratch for a call; `extra` is the pCN moves (WS_JITTER,
    WS_TEMPERED) or the checkpoint interval (WS_NUDGE_GRAD, WS_NUDGE)."""
    mc = model.c() if model is not None else None
    return int(lib().sch_workspace_bytes(which, C.byref(mc) if mc is not None else None,
                                         n_particles, n_steps, extra))


def workspace(which: int, model: Model | None, n_particles: int, n_steps: int = 0,
              extra: int = 0, device="cuda") -> torch.Tensor:
    nb = workspace_bytes(which, model, n_particles, n_steps, extra)
    if nb <= 0:
        raise SchError(SCH_E_ARG, "invalid workspace request")
    return torch.empty(nb, dtype=torch.uint8, device=device)


# --------------------------------------------------------------------------- calls
def sch_draw_increments(seed: int, cycle: int, temper_k: int, tag: int, dW: torch.Tensor,
                        dt: float):
    n, s, q = dW.shape
    r = SchRngC(seed, cycle, temper_k)
    _check(lib().sch_draw_increments(C.byref(r), tag, n, s, q, dt, _dev(dW, name="dW"),
                                     _stream()))


def sch_philox_blocks(seed: int, ctr: torch.Tensor, out: torch.Tensor):
    """ctr, out: int32 tensors [n][4] holding uint32 bit patterns."""
    _check(lib().sch_philox_blocks(seed, ctr.shape[0], _dev(ctr, torch.int32, "ctr"),
                                   _dev(out, torch.int32, "out"), _stream()))


def sch_velocity(model: Model, m: torch.Tensor, u: torch.Tensor):
    mc = model.c()
    _state(model, m.shape[0], m=m, u=u)
    _check(lib().sch_velocity(C.byref(mc), m.shape[0], _dev(m, name="m"), _dev(u, name="u"),
                              _stream()))


def sch_init_momentum(model: Model, u: torch.Tensor, m: torch.Tensor):
    mc = model.c()
    _state(model, u.shape[0], u=u, m=m)
    _check(lib().sch_init_momentum(C.byref(mc), u.shape[0], _dev(u, name="u"), _dev(m, name="m"),
                                   _stream()))


def sch_ensemble_step(model: Model, m: torch.Tensor, u: torch.Tensor, dW: torch.Tensor,
                      dLambda: torch.Tensor | None = None, status: torch.Tensor | None = None,
                      iters: torch.Tensor | None = None):
    mc = model.c()
    n, s = dW.shape[0], dW.shape[1]
    _state(model, n, m=m, u=u)
    _inc(n, s, model.n_modes, dW=dW, dLambda=dLambda)
    _vec(n, status=status, iters=iters)
    _check(lib().sch_ensemble_step(C.byref(mc), n, s, _dev(m, name="m"), _dev(u, name="u"),
                                   _dev(dW, name="dW"), _dev(dLambda, name="dLambda"),
                                   _dev(status, torch.int32, "status"),
                                   _dev(iters, torch.int32, "iters"), _stream()))


def sch_observe(model: Model, u: torch.Tensor, out: torch.Tensor):
    mc = model.c()
    _state(model, u.shape[0], u=u)
    _shape(out, (u.shape[0], out.shape[-1]), "out")
    _check(lib().sch_observe(C.byref(mc), out.shape[-1], u.shape[0], _dev(u, name="u"),
                             _dev(out, name="out"), _stream()))


def sch_loglik(model: Model, obs: Obs, u: torch.Tensor, phi: torch.Tensor):
    mc, oc = model.c(), obs.c()
    _state(model, u.shape[0], u=u)
    _vec(u.shape[0], phi=phi)
    _check(lib().sch_loglik(C.byref(mc), C.byref(oc), u.shape[0], _dev(u, name="u"),
                            _dev(phi, name="phi"), _stream()))


def sch_temper_ess(phi: torch.Tensor, theta: torch.Tensor, ess_threshold: float, n_bisect: int,
                   dtheta: torch.Tensor, w: torch.Tensor, ess: torch.Tensor,
                   logw_extra: torch.Tensor | None = None, logw_out: torch.Tensor | None = None):
    n = phi.numel()
    _vec(n, w=w, logw_extra=logw_extra, logw_out=logw_out)
    _at_least(theta, 1, "theta")
    _at_least(dtheta, 1, "dtheta")
    _at_least(ess, 1, "ess")
    _check(lib().sch_temper_ess(phi.numel(), _dev(phi, name="phi"),
                                _dev(logw_extra, name="logw_extra"), _dev(theta, name="theta"),
                                ess_threshold, n_bisect, _dev(dtheta, name="dtheta"),
                                _dev(w, name="w"), _dev(logw_out, name="logw_out"),
                                _dev(ess, name="ess"), _stream()))


def sch_resample(w: torch.Tensor, u0: torch.Tensor, idx: torch.Tensor, workspace: torch.Tensor,
                 cond_ess: torch.Tensor | None = None, cond_threshold: float = 0.0,
                 degenerate: torch.Tensor | None = None):
    n = w.numel()
    _vec(n, idx=idx)
    _at_least(u0, 1, "u0")
    _at_least(cond_ess, 1, "cond_ess")
    _ws(workspace, workspace_bytes(WS_RESAMPLE, None, n))
    _check(lib().sch_resample(w.numel(), _dev(w, name="w"), _dev(u0, name="u0"),
                              _dev(cond_ess, name="cond_ess"), cond_threshold,
                              _dev(idx, torch.int32, "idx"), _dev(degenerate, torch.int32,
                                                                 "degenerate"),
                              _dev(workspace, torch.uint8, "workspace"), _stream()))


def sch_gather(idx: torch.Tensor, src: torch.Tensor, dst: torch.Tensor):
    n = idx.numel()
    row = src.numel() // src.shape[0]
    if dst.shape[1:] != src.shape[1:] or dst.shape[0] != n:
        raise SchError(SCH_E_SHAPE, f"dst {tuple(dst.shape)} must be [{n}] + {tuple(src.shape[1:])}")
    _check(lib().sch_gather(n, row, _dev(idx, torch.int32, "idx"), _dev(src, name="src"),
                            _dev(dst, name="dst"), _stream()))


def sch_jitter_pcn(model: Model, obs: Obs, seed: int, cycle: int, temper_k: int,
                   m0: torch.Tensor, u0: torch.Tensor, dW: torch.Tensor, phi: torch.Tensor,
                   m_end: torch.Tensor, u_end: torch.Tensor, theta: torch.Tensor, rho: float,
                   n_jitter: int, n_accept: torch.Tensor | None = None,
                   workspace: torch.Tensor | None = None, dLambda: torch.Tensor | None = None):
    """pCN moves of dW; with dLambda (fixed controls) phi holds the nudged
    potential J."""
    mc, oc = model.c(), obs.c()
    r = SchRngC(seed, cycle, temper_k)
    n, s = dW.shape[0], dW.shape[1]
    _state(model, n, m0=m0, u0=u0, m_end=m_end, u_end=u_end)
    _inc(n, s, model.n_modes, dW=dW, dLambda=dLambda)
    _vec(n, phi=phi, n_accept=n_accept)
    _at_least(theta, 1, "theta")
    if workspace is None:
        workspace = globals()["workspace"](WS_JITTER, model, n, s, n_jitter)
    _ws(workspace, workspace_bytes(WS_JITTER, model, n, s, n_jitter))
    _check(lib().sch_jitter_pcn(C.byref(mc), C.byref(oc), C.byref(r), n, s, _dev(m0, name="m0"),
                                _dev(u0, name="u0"), _dev(dW, name="dW"),
                                _dev(dLambda, name="dLambda"), _dev(phi, name="phi"),
                                _dev(m_end, name="m_end"), _dev(u_end, name="u_end"),
                                _dev(theta, name="theta"), rho, n_jitter,
                                _dev(n_accept, torch.int32, "n_accept"),
                                _dev(workspace, torch.uint8, "workspace"), _stream()))


def sch_jitter_pcn_noalloc(model: Model, obs: Obs, seed: int, cycle: int, temper_k: int,
                           m0: torch.Tensor, u0: torch.Tensor, dW: torch.Tensor,
                           phi: torch.Tensor, m_end: torch.Tensor, u_end: torch.Tensor,
                           theta: torch.Tensor, rho: float, n_jitter: int,
                           n_accept: torch.Tensor | None = None,
                           dLambda: torch.Tensor | None = None):
    """sch_jitter_pcn with its proposal draws in the library's own device
    array (no workspace; at most sch_jitter_pcn_noalloc_max_bytes())."""
    mc, oc = model.c(), obs.c()
    r = SchRngC(seed, cycle, temper_k)
    n, s = dW.shape[0], dW.shape[1]
    _state(model, n, m0=m0, u0=u0, m_end=m_end, u_end=u_end)
    _inc(n, s, model.n_modes, dW=dW, dLambda=dLambda)
    _vec(n, phi=phi, n_accept=n_accept)
    _at_least(theta, 1, "theta")
    _check(lib().sch_jitter_pcn_noalloc(C.byref(mc), C.byref(oc), C.byref(r), n, s,
                                        _dev(m0, name="m0"), _dev(u0, name="u0"),
                                        _dev(dW, name="dW"), _dev(dLambda, name="dLambda"),
                                        _dev(phi, name="phi"), _dev(m_end, name="m_end"),
                                        _dev(u_end, name="u_end"), _dev(theta, name="theta"),
                                        rho, n_jitter, _dev(n_accept, torch.int32, "n_accept"),
                                        _stream()))


def sch_pf_bootstrap_cycle(model: Model, obs: Obs, seed: int, cycle: int, m: torch.Tensor,
                           u: torch.Tensor, logw: torch.Tensor, n_steps: int, ess_frac: float,
                           workspace: torch.Tensor) -> dict:
    mc, oc = model.c(), obs.c()
    n = m.shape[0]
    _state(model, n, m=m, u=u)
    _vec(n, logw=logw)
    _ws(workspace, workspace_bytes(WS_BOOTSTRAP, model, n, n_steps))
    st = SchCycleStats()
    _check(lib().sch_pf_bootstrap_cycle(C.byref(mc), C.byref(oc), seed, cycle, m.shape[0],
                                        n_steps, ess_frac, _dev(m, name="m"), _dev(u, name="u"),
                                        _dev(logw, name="logw"),
                                        _dev(workspace, torch.uint8, "workspace"), C.byref(st),
                                        _stream()))
    return st.as_dict()


def sch_pf_tempered_cycle(model: Model, obs: Obs, seed: int, cycle: int, m: torch.Tensor,
                          u: torch.Tensor, n_steps: int, ess_threshold: float, n_bisect: int,
                          rho: float, n_jitter: int, max_temper: int,
                          workspace: torch.Tensor) -> dict:
    mc, oc = model.c(), obs.c()
    n = m.shape[0]
    _state(model, n, m=m, u=u)
    _ws(workspace, workspace_bytes(WS_TEMPERED, model, n, n_steps, n_jitter))
    st = SchCycleStats()
    _check(lib().sch_pf_tempered_cycle(C.byref(mc), C.byref(oc), seed, cycle, m.shape[0],
                                       n_steps, ess_threshold, n_bisect, rho, n_jitter,
                                       max_temper, _dev(m, name="m"), _dev(u, name="u"),
                                       _dev(workspace, torch.uint8, "workspace"), C.byref(st),
                                       _stream()))
    return st.as_dict()


# --------------------------------------------------------------------------- Matern noise
@dataclass
class Matern:
    """Matern-type noise of section 2 (eq. noise_solve2): k solves with
    M + kappa^-2 K on the DG0 white noise, amplitude eta."""
    kappa: float = 1.0
    eta: float = 1.0
    k: int = 3

    def c(self) -> SchMaternC:
        return SchMaternC(self.kappa, self.eta, self.k)


def sch_matern_field(model: Model, mt: Matern, dWc: torch.Tensor, dU: torch.Tensor):
    mc, tc = model.c(), mt.c()
    _state(model, dWc.shape[0], dWc=dWc, dU=dU)
    _check(lib().sch_matern_field(C.byref(mc), C.byref(tc), dWc.shape[0], _dev(dWc, name="dWc"),
                                  _dev(dU, name="dU"), _stream()))


def sch_ensemble_step_matern(model: Model, mt: Matern, m: torch.Tensor, u: torch.Tensor,
                             dWc: torch.Tensor, status: torch.Tensor | None = None,
                             iters: torch.Tensor | None = None):
    mc, tc = model.c(), mt.c()
    n, s = dWc.shape[0], dWc.shape[1]
    _state(model, n, m=m, u=u)
    _inc(n, s, model.nx, dWc=dWc)
    _vec(n, status=status, iters=iters)
    _check(lib().sch_ensemble_step_matern(C.byref(mc), C.byref(tc), n, s, _dev(m, name="m"),
                                          _dev(u, name="u"), _dev(dWc, name="dWc"),
                                          _dev(status, torch.int32, "status"),
                                          _dev(iters, torch.int32, "iters"), _stream()))


def matern_workspace(which: int, model: Model, n_particles: int, n_steps: int, extra: int,
                     device="cuda") -> torch.Tensor:
    """Scratch of the Matern-noise calls; extra is n_jitter (jitter and
    cycles) or ckpt_every (WS_NUDGE_GRAD, WS_NUDGE)."""
    return torch.empty(matern_workspace_bytes(which, model, n_particles, n_steps, extra),
                       dtype=torch.uint8, device=device)


def matern_workspace_bytes(which: int, model: Model, n_particles: int, n_steps: int,
                           extra: int) -> int:
    mc = model.c()
    nb = int(lib().sch_matern_workspace_bytes(which, C.byref(mc), n_particles, n_steps, extra))
    if nb <= 0:
        raise SchError(SCH_E_ARG, "invalid workspace request")
    return nb


def sch_jitter_pcn_matern(model: Model, mt: Matern, obs: Obs, seed: int, cycle: int,
                          temper_k: int, m0: torch.Tensor, u0: torch.Tensor, dWc: torch.Tensor,
                          phi: torch.Tensor, m_end: torch.Tensor, u_end: torch.Tensor,
                          theta: torch.Tensor, rho: float, n_jitter: int,
                          n_accept: torch.Tensor | None = None,
                          workspace: torch.Tensor | None = None):
    mc, tc, oc = model.c(), mt.c(), obs.c()
    r = SchRngC(seed, cycle, temper_k)
    n, s = dWc.shape[0], dWc.shape[1]
    _state(model, n, m0=m0, u0=u0, m_end=m_end, u_end=u_end)
    _inc(n, s, model.nx, dWc=dWc)
    _vec(n, phi=phi, n_accept=n_accept)
    _at_least(theta, 1, "theta")
    if workspace is None:
        workspace = matern_workspace(WS_JITTER, model, n, s, n_jitter)
    _ws(workspace, matern_workspace_bytes(WS_JITTER, model, n, s, n_jitter))
    _check(lib().sch_jitter_pcn_matern(C.byref(mc), C.byref(tc), C.byref(oc), C.byref(r), n, s,
                                       _dev(m0, name="m0"), _dev(u0, name="u0"),
                                       _dev(dWc, name="dWc"), _dev(phi, name="phi"),
                                       _dev(m_end, name="m_end"), _dev(u_end, name="u_end"),
                                       _dev(theta, name="theta"), rho, n_jitter,
                                       _dev(n_accept, torch.int32, "n_accept"),
                                       _dev(workspace, torch.uint8, "workspace"), _stream()))


def sch_jitter_pcn_matern_ctrl(model: Model, mt: Matern, obs: Obs, seed: int, cycle: int,
                               temper_k: int, m0: torch.Tensor, u0: torch.Tensor,
                               dWc: torch.Tensor, dLambdac: torch.Tensor, J: torch.Tensor,
                               m_end: torch.Tensor, u_end: torch.Tensor, theta: torch.Tensor,
                               rho: float, n_jitter: int, n_accept: torch.Tensor | None = None,
                               workspace: torch.Tensor | None = None):
    """sch_jitter_pcn_matern with the per-cell controls dLambdac held fixed;
    J holds the nudged potentials."""
    mc, tc, oc = model.c(), mt.c(), obs.c()
    r = SchRngC(seed, cycle, temper_k)
    n, s = dWc.shape[0], dWc.shape[1]
    _state(model, n, m0=m0, u0=u0, m_end=m_end, u_end=u_end)
    _inc(n, s, model.nx, dWc=dWc, dLambdac=dLambdac)
    _vec(n, J=J, n_accept=n_accept)
    _at_least(theta, 1, "theta")
    if workspace is None:
        workspace = matern_workspace(WS_JITTER, model, n, s, n_jitter)
    _ws(workspace, matern_workspace_bytes(WS_JITTER, model, n, s, n_jitter))
    _check(lib().sch_jitter_pcn_matern_ctrl(C.byref(mc), C.byref(tc), C.byref(oc), C.byref(r), n,
                                            s, _dev(m0, name="m0"), _dev(u0, name="u0"),
                                            _dev(dWc, name="dWc"),
                                            _dev(dLambdac, name="dLambdac"), _dev(J, name="J"),
                                            _dev(m_end, name="m_end"), _dev(u_end, name="u_end"),
                                            _dev(theta, name="theta"), rho, n_jitter,
                                            _dev(n_accept, torch.int32, "n_accept"),
                                            _dev(workspace, torch.uint8, "workspace"),
                                            _stream()))


def sch_pf_tempered_cycle_matern(model: Model, mt: Matern, obs: Obs, seed: int, cycle: int,
                                 m: torch.Tensor, u: torch.Tensor, n_steps: int,
                                 ess_threshold: float, n_bisect: int, rho: float, n_jitter: int,
                                 max_temper: int, workspace: torch.Tensor) -> dict:
    mc, tc, oc = model.c(), mt.c(), obs.c()
    n = m.shape[0]
    _state(model, n, m=m, u=u)
    _ws(workspace, matern_workspace_bytes(WS_TEMPERED, model, n, n_steps, n_jitter))
    st = SchCycleStats()
    _check(lib().sch_pf_tempered_cycle_matern(C.byref(mc), C.byref(tc), C.byref(oc), seed, cycle,
                                              m.shape[0], n_steps, ess_threshold, n_bisect, rho,
                                              n_jitter, max_temper, _dev(m, name="m"),
                                              _dev(u, name="u"),
                                              _dev(workspace, torch.uint8, "workspace"),
                                              C.byref(st), _stream()))
    return st.as_dict()


def sch_pf_bootstrap_cycle_matern(model: Model, mt: Matern, obs: Obs, seed: int, cycle: int,
                                  m: torch.Tensor, u: torch.Tensor, logw: torch.Tensor,
                                  n_steps: int, ess_frac: float, workspace: torch.Tensor) -> dict:
    mc, tc, oc = model.c(), mt.c(), obs.c()
    n = m.shape[0]
    _state(model, n, m=m, u=u)
    _vec(n, logw=logw)
    _ws(workspace, matern_workspace_bytes(WS_BOOTSTRAP, model, n, n_steps, 0))
    st = SchCycleStats()
    _check(lib().sch_pf_bootstrap_cycle_matern(C.byref(mc), C.byref(tc), C.byref(oc), seed,
                                               cycle, m.shape[0], n_steps, ess_frac,
                                               _dev(m, name="m"), _dev(u, name="u"),
                                               _dev(logw, name="logw"),
                                               _dev(workspace, torch.uint8, "workspace"),
                                               C.byref(st), _stream()))
    return st.as_dict()


# --------------------------------------------------------------------------- pCN Langevin
def pcnl_workspace(which: int, model: Model, n_particles: int, n_steps: int, n_jitter: int,
                   ckpt_every: int = 8, device="cuda") -> torch.Tensor:
    return torch.empty(pcnl_workspace_bytes(which, model, n_particles, n_steps, n_jitter,
                                            ckpt_every), dtype=torch.uint8, device=device)


def pcnl_workspace_bytes(which: int, model: Model, n_particles: int, n_steps: int,
                         n_jitter: int, ckpt_every: int = 8) -> int:
    mc = model.c()
    nb = int(lib().sch_pcnl_workspace_bytes(which, C.byref(mc), n_particles, n_steps, n_jitter,
                                            ckpt_every))
    if nb <= 0:
        raise SchError(SCH_E_ARG, "invalid workspace request")
    return nb


def sch_jitter_pcnl(model: Model, obs: Obs, seed: int, cycle: int, temper_k: int,
                    m0: torch.Tensor, u0: torch.Tensor, dW: torch.Tensor, phi: torch.Tensor,
                    m_end: torch.Tensor, u_end: torch.Tensor, theta: torch.Tensor, rho: float,
                    n_jitter: int, ckpt_every: int = 8, n_accept: torch.Tensor | None = None,
                    workspace: torch.Tensor | None = None):
    mc, oc = model.c(), obs.c()
    r = SchRngC(seed, cycle, temper_k)
    n, s = dW.shape[0], dW.shape[1]
    _state(model, n, m0=m0, u0=u0, m_end=m_end, u_end=u_end)
    _inc(n, s, model.n_modes, dW=dW)
    _vec(n, phi=phi, n_accept=n_accept)
    _at_least(theta, 1, "theta")
    if workspace is None:
        workspace = pcnl_workspace(WS_JITTER, model, n, s, n_jitter, ckpt_every)
    _ws(workspace, pcnl_workspace_bytes(WS_JITTER, model, n, s, n_jitter, ckpt_every))
    _check(lib().sch_jitter_pcnl(C.byref(mc), C.byref(oc), C.byref(r), n, s, _dev(m0, name="m0"),
                                 _dev(u0, name="u0"), _dev(dW, name="dW"), _dev(phi, name="phi"),
                                 _dev(m_end, name="m_end"), _dev(u_end, name="u_end"),
                                 _dev(theta, name="theta"), rho, n_jitter, ckpt_every,
                                 _dev(n_accept, torch.int32, "n_accept"),
                                 _dev(workspace, torch.uint8, "workspace"), _stream()))


def sch_pf_tempered_cycle_pcnl(model: Model, obs: Obs, seed: int, cycle: int, m: torch.Tensor,
                               u: torch.Tensor, n_steps: int, ess_threshold: float,
                               n_bisect: int, rho: float, n_jitter: int, max_temper: int,
                               workspace: torch.Tensor, ckpt_every: int = 8) -> dict:
    mc, oc = model.c(), obs.c()
    n = m.shape[0]
    _state(model, n, m=m, u=u)
    _ws(workspace, pcnl_workspace_bytes(WS_TEMPERED, model, n, n_steps, n_jitter, ckpt_every))
    st = SchCycleStats()
    _check(lib().sch_pf_tempered_cycle_pcnl(C.byref(mc), C.byref(oc), seed, cycle, m.shape[0],
                                            n_steps, ess_threshold, n_bisect, rho, n_jitter,
                                            max_temper, ckpt_every, _dev(m, name="m"),
                                            _dev(u, name="u"),
                                            _dev(workspace, torch.uint8, "workspace"),
                                            C.byref(st), _stream()))
    return st.as_dict()


# --------------------------------------------------------------------------- Hybrid Monte Carlo
def hmc_workspace(which: int, model: Model, n_particles: int, n_steps: int, n_jitter: int,
                  ckpt_every: int = 8, device="cuda") -> torch.Tensor:
    return torch.empty(hmc_workspace_bytes(which, model, n_particles, n_steps, n_jitter,
                                           ckpt_every), dtype=torch.uint8, device=device)


def hmc_workspace_bytes(which: int, model: Model, n_particles: int, n_steps: int,
                        n_jitter: int, ckpt_every: int = 8) -> int:
    mc = model.c()
    nb = int(lib().sch_hmc_workspace_bytes(which, C.byref(mc), n_particles, n_steps, n_jitter,
                                           ckpt_every))
    if nb <= 0:
        raise SchError(SCH_E_ARG, "invalid workspace request")
    return nb


def sch_jitter_hmc(model: Model, obs: Obs, seed: int, cycle: int, temper_k: int,
                   m0: torch.Tensor, u0: torch.Tensor, dW: torch.Tensor, phi: torch.Tensor,
                   m_end: torch.Tensor, u_end: torch.Tensor, theta: torch.Tensor, h: float,
                   n_leap: int, n_jitter: int, ckpt_every: int = 8,
                   n_accept: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
    mc, oc = model.c(), obs.c()
    r = SchRngC(seed, cycle, temper_k)
    n, s = dW.shape[0], dW.shape[1]
    _state(model, n, m0=m0, u0=u0, m_end=m_end, u_end=u_end)
    _inc(n, s, model.n_modes, dW=dW)
    _vec(n, phi=phi, n_accept=n_accept)
    _at_least(theta, 1, "theta")
    if workspace is None:
        workspace = hmc_workspace(WS_JITTER, model, n, s, n_jitter, ckpt_every)
    _ws(workspace, hmc_workspace_bytes(WS_JITTER, model, n, s, n_jitter, ckpt_every))
    _check(lib().sch_jitter_hmc(C.byref(mc), C.byref(oc), C.byref(r), n, s, _dev(m0, name="m0"),
                                _dev(u0, name="u0"), _dev(dW, name="dW"), _dev(phi, name="phi"),
                                _dev(m_end, name="m_end"), _dev(u_end, name="u_end"),
                                _dev(theta, name="theta"), h, n_leap, n_jitter, ckpt_every,
                                _dev(n_accept, torch.int32, "n_accept"),
                                _dev(workspace, torch.uint8, "workspace"), _stream()))


def sch_pf_tempered_cycle_hmc(model: Model, obs: Obs, seed: int, cycle: int, m: torch.Tensor,
                              u: torch.Tensor, n_steps: int, ess_threshold: float,
                              n_bisect: int, h: float, n_leap: int, n_jitter: int,
                              max_temper: int, workspace: torch.Tensor,
                              ckpt_every: int = 8) -> dict:
    mc, oc = model.c(), obs.c()
    n = m.shape[0]
    _state(model, n, m=m, u=u)
    _ws(workspace, hmc_workspace_bytes(WS_TEMPERED, model, n, n_steps, n_jitter, ckpt_every))
    st = SchCycleStats()
    _check(lib().sch_pf_tempered_cycle_hmc(C.byref(mc), C.byref(oc), seed, cycle, m.shape[0],
                                           n_steps, ess_threshold, n_bisect, h, n_leap, n_jitter,
                                           max_temper, ckpt_every, _dev(m, name="m"),
                                           _dev(u, name="u"),
                                           _dev(workspace, torch.uint8, "workspace"),
                                           C.byref(st), _stream()))
    return st.as_dict()


# --------------------------------------------------------------------------- section 4
def sch_paper_init(model: Model, seed: int, u: torch.Tensor):
    """Initial velocities of eq. init_solve for the rows of u [n][nx]."""
    mc = model.c()
    _state(model, u.shape[0], u=u)
    _check(lib().sch_paper_init(C.byref(mc), seed, u.shape[0], _dev(u, name="u"), _stream()))


def sch_ensemble_stats(u: torch.Tensor, ua: torch.Tensor, workspace: torch.Tensor | None = None,
                       out: torch.Tensor | None = None) -> torch.Tensor:
    """(EMRE, RB, RES) of the ensemble u [n][nx] against the truth ua [nx], on the GPU."""
    n, nx = u.shape
    _shape(ua, (nx,), "ua")
    if workspace is None:
        workspace = torch.empty(nx + 2 * n, dtype=torch.float64, device=u.device)
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=u.device)
    _at_least(workspace, nx + 2 * n, "workspace")
    _at_least(out, 3, "out")
    _check(lib().sch_ensemble_stats(n, nx, _dev(u, name="u"), _dev(ua, name="ua"),
                                    _dev(workspace, name="workspace"), _dev(out, name="out"),
                                    _stream()))
    return out


def sch_nudge_grad(model: Model, obs: Obs, m0: torch.Tensor, u0: torch.Tensor,
                   dW: torch.Tensor | None, dLambda: torch.Tensor | None, J: torch.Tensor,
                   grad: torch.Tensor, ckpt_every: int = 8, status: torch.Tensor | None = None,
                   workspace: torch.Tensor | None = None):
    """J [n] and dJ/d(dLambda) [n][n_steps][Q]; the window length is grad.shape[1]."""
    mc, oc = model.c(), obs.c()
    n, s = grad.shape[0], grad.shape[1]
    _state(model, n, m0=m0, u0=u0)
    _inc(n, s, model.n_modes, grad=grad, dW=dW, dLambda=dLambda)
    _vec(n, J=J, status=status)
    if workspace is None:
        workspace = globals()["workspace"](WS_NUDGE_GRAD, model, n, s, ckpt_every)
    _ws(workspace, workspace_bytes(WS_NUDGE_GRAD, model, n, s, ckpt_every))
    _check(lib().sch_nudge_grad(C.byref(mc), C.byref(oc), n, s, _dev(m0, name="m0"),
                                _dev(u0, name="u0"), _dev(dW, name="dW"),
                                _dev(dLambda, name="dLambda"), ckpt_every, _dev(J, name="J"),
                                _dev(grad, name="grad"), _dev(status, torch.int32, "status"),
                                _dev(workspace, torch.uint8, "workspace"), _stream()))


LBFGS_GTOL, LBFGS_MAX_ITER, LBFGS_MEM, LBFGS_MAX_BACK = 1e-8, 30, 8, 30


def sch_nudge_run(model: Model, obs: Obs, m: torch.Tensor, u: torch.Tensor, dW: torch.Tensor,
                  dLambda: torch.Tensor, logG: torch.Tensor, warm_start: bool = False,
                  gtol: float = LBFGS_GTOL, max_iter: int = LBFGS_MAX_ITER,
                  mem: int = LBFGS_MEM, max_back: int = LBFGS_MAX_BACK, ckpt_every: int = 8,
                  lbfgs_status: torch.Tensor | None = None, iters: torch.Tensor | None = None,
                  evals: torch.Tensor | None = None, status: torch.Tensor | None = None,
                  workspace: torch.Tensor | None = None):
    mc, oc = model.c(), obs.c()
    n, s = dW.shape[0], dW.shape[1]
    _state(model, n, m=m, u=u)
    _inc(n, s, model.n_modes, dW=dW, dLambda=dLambda)
    _vec(n, logG=logG, lbfgs_status=lbfgs_status, iters=iters, evals=evals, status=status)
    if workspace is None:
        workspace = globals()["workspace"](WS_NUDGE, model, n, s, ckpt_every)
    _ws(workspace, workspace_bytes(WS_NUDGE, model, n, s, ckpt_every))
    opts = SchLbfgsOpts(gtol, max_iter, mem, max_back)
    _check(lib().sch_nudge_run(C.byref(mc), C.byref(oc), n, s, _dev(m, name="m"),
                               _dev(u, name="u"), _dev(dW, name="dW"),
                               _dev(dLambda, name="dLambda"), 1 if warm_start else 0,
                               C.byref(opts), ckpt_every, _dev(logG, name="logG"),
                               _dev(lbfgs_status, torch.int32, "lbfgs_status"),
                               _dev(iters, torch.int32, "iters"),
                               _dev(evals, torch.int32, "evals"),
                               _dev(status, torch.int32, "status"),
                               _dev(workspace, torch.uint8, "workspace"), _stream()))


def sch_nudge_grad_matern(model: Model, mt: Matern, obs: Obs, m0: torch.Tensor,
                          u0: torch.Tensor, dWc: torch.Tensor | None,
                          dLambdac: torch.Tensor | None, J: torch.Tensor, grad: torch.Tensor,
                          ckpt_every: int = 8, status: torch.Tensor | None = None,
                          workspace: torch.Tensor | None = None):
    """sch_nudge_grad with the Matern-type noise: controls and gradient per
    cell, [n][n_steps][nx]; the window length is grad.shape[1]."""
    mc, tc, oc = model.c(), mt.c(), obs.c()
    n, s = grad.shape[0], grad.shape[1]
    _state(model, n, m0=m0, u0=u0)
    _inc(n, s, model.nx, grad=grad, dWc=dWc, dLambdac=dLambdac)
    _vec(n, J=J, status=status)
    if workspace is None:
        workspace = matern_workspace(WS_NUDGE_GRAD, model, n, s, ckpt_every)
    _ws(workspace, matern_workspace_bytes(WS_NUDGE_GRAD, model, n, s, ckpt_every))
    _check(lib().sch_nudge_grad_matern(C.byref(mc), C.byref(tc), C.byref(oc), n, s,
                                       _dev(m0, name="m0"), _dev(u0, name="u0"),
                                       _dev(dWc, name="dWc"), _dev(dLambdac, name="dLambdac"),
                                       ckpt_every, _dev(J, name="J"), _dev(grad, name="grad"),
                                       _dev(status, torch.int32, "status"),
                                       _dev(workspace, torch.uint8, "workspace"), _stream()))


def sch_nudge_run_matern(model: Model, mt: Matern, obs: Obs, m: torch.Tensor, u: torch.Tensor,
                         dWc: torch.Tensor, dLambdac: torch.Tensor, logG: torch.Tensor,
                         warm_start: bool = False, gtol: float = LBFGS_GTOL,
                         max_iter: int = LBFGS_MAX_ITER, mem: int = LBFGS_MEM,
                         max_back: int = LBFGS_MAX_BACK, ckpt_every: int = 8,
                         lbfgs_status: torch.Tensor | None = None,
                         iters: torch.Tensor | None = None, evals: torch.Tensor | None = None,
                         status: torch.Tensor | None = None,
                         workspace: torch.Tensor | None = None):
    """sch_nudge_run with the Matern-type noise: one control per cell."""
    mc, tc, oc = model.c(), mt.c(), obs.c()
    n, s = dWc.shape[0], dWc.shape[1]
    _state(model, n, m=m, u=u)
    _inc(n, s, model.nx, dWc=dWc, dLambdac=dLambdac)
    _vec(n, logG=logG, lbfgs_status=lbfgs_status, iters=iters, evals=evals, status=status)
    if workspace is None:
        workspace = matern_workspace(WS_NUDGE, model, n, s, ckpt_every)
    _ws(workspace, matern_workspace_bytes(WS_NUDGE, model, n, s, ckpt_every))
    opts = SchLbfgsOpts(gtol, max_iter, mem, max_back)
    _check(lib().sch_nudge_run_matern(C.byref(mc), C.byref(tc), C.byref(oc), n, s,
                                      _dev(m, name="m"), _dev(u, name="u"),
                                      _dev(dWc, name="dWc"), _dev(dLambdac, name="dLambdac"),
                                      1 if warm_start else 0, C.byref(opts), ckpt_every,
                                      _dev(logG, name="logG"),
                                      _dev(lbfgs_status, torch.int32, "lbfgs_status"),
                                      _dev(iters, torch.int32, "iters"),
                                      _dev(evals, torch.int32, "evals"),
                                      _dev(status, torch.int32, "status"),
                                      _dev(workspace, torch.uint8, "workspace"), _stream()))


def nudged_workspace(model: Model, n_particles: int, n_steps: int, n_jitter: int,
                     ckpt_every: int = 8, device="cuda") -> torch.Tensor:
    return torch.empty(nudged_workspace_bytes(model, n_particles, n_steps, n_jitter, ckpt_every),
                       dtype=torch.uint8, device=device)


def nudged_workspace_bytes(model: Model, n_particles: int, n_steps: int, n_jitter: int,
                           ckpt_every: int = 8) -> int:
    mc = model.c()
    nb = int(lib().sch_nudged_workspace_bytes(C.byref(mc), n_particles, n_steps, n_jitter,
                                              ckpt_every))
    if nb <= 0:
        raise SchError(SCH_E_ARG, "invalid workspace request")
    return nb


def sch_pf_nudged_cycle(model: Model, obs: Obs, seed: int, cycle: int, m: torch.Tensor,
                        u: torch.Tensor, dLambda: torch.Tensor, n_steps: int,
                        ess_threshold: float, n_bisect: int, rho: float, n_jitter: int,
                        max_temper: int, workspace: torch.Tensor, gtol: float = LBFGS_GTOL,
                        max_iter: int = LBFGS_MAX_ITER, mem: int = LBFGS_MEM,
                        max_back: int = LBFGS_MAX_BACK, ckpt_every: int = 8) -> dict:
    mc, oc = model.c(), obs.c()
    n = m.shape[0]
    _state(model, n, m=m, u=u)
    _inc(n, n_steps, model.n_modes, dLambda=dLambda)
    _ws(workspace, nudged_workspace_bytes(model, n, n_steps, n_jitter, ckpt_every))
    st = SchCycleStats()
    opts = SchLbfgsOpts(gtol, max_iter, mem, max_back)
    _check(lib().sch_pf_nudged_cycle(C.byref(mc), C.byref(oc), seed, cycle, m.shape[0], n_steps,
                                     ess_threshold, n_bisect, rho, n_jitter, max_temper,
                                     C.byref(opts), ckpt_every, _dev(m, name="m"),
                                     _dev(u, name="u"), _dev(dLambda, name="dLambda"),
                                     _dev(workspace, torch.uint8, "workspace"), C.byref(st),
                                     _stream()))
    return st.as_dict()


def nudged_workspace_matern(model: Model, n_particles: int, n_steps: int, n_jitter: int,
                            ckpt_every: int = 8, device="cuda") -> torch.Tensor:
    return torch.empty(nudged_workspace_bytes_matern(model, n_particles, n_steps, n_jitter,
                                                     ckpt_every),
                       dtype=torch.uint8, device=device)


NUDGE_KEEP, NUDGE_FROM_GIVEN, NUDGE_FROM_ZERO = 0, 1, 2


def sch_pf_nudged_cycle_warm(model: Model, obs: Obs, seed: int, cycle: int, m: torch.Tensor,
                             u: torch.Tensor, dLambda: torch.Tensor, mode: torch.Tensor,
                             n_steps: int, ess_threshold: float, n_bisect: int, rho: float,
                             n_jitter: int, max_temper: int, workspace: torch.Tensor,
                             gtol: float = LBFGS_GTOL, max_iter: int = LBFGS_MAX_ITER,
                             mem: int = LBFGS_MEM, max_back: int = LBFGS_MAX_BACK,
                             ckpt_every: int = 8) -> dict:
    """The nudged filter from given start controls dLambda (in/out) with a
    per-particle start mode (NUDGE_KEEP, NUDGE_FROM_GIVEN, NUDGE_FROM_ZERO)."""
    n = m.shape[0]
    _state(model, n, m=m, u=u)
    _inc(n, n_steps, model.n_modes, dLambda=dLambda)
    _vec(n, mode=mode)
    _ws(workspace, nudged_workspace_bytes(model, n, n_steps, n_jitter, ckpt_every))
    mc, oc = model.c(), obs.c()
    st = SchCycleStats()
    opts = SchLbfgsOpts(gtol, max_iter, mem, max_back)
    _check(lib().sch_pf_nudged_cycle_warm(C.byref(mc), C.byref(oc), seed, cycle, n, n_steps,
                                          ess_threshold, n_bisect, rho, n_jitter, max_temper,
                                          C.byref(opts), ckpt_every, _dev(m, name="m"),
                                          _dev(u, name="u"), _dev(dLambda, name="dLambda"),
                                          _dev(mode, torch.int32, "mode"),
                                          _dev(workspace, torch.uint8, "workspace"), C.byref(st),
                                          _stream()))
    return st.as_dict()


def nudged_workspace_bytes_matern(model: Model, n_particles: int, n_steps: int, n_jitter: int,
                                  ckpt_every: int = 8) -> int:
    mc = model.c()
    nb = int(lib().sch_nudged_workspace_bytes_matern(C.byref(mc), n_particles, n_steps,
                                                     n_jitter, ckpt_every))
    if nb <= 0:
        raise SchError(SCH_E_ARG, "invalid workspace request")
    return nb


def sch_pf_nudged_cycle_matern(model: Model, mt: Matern, obs: Obs, seed: int, cycle: int,
                               m: torch.Tensor, u: torch.Tensor, dLambdac: torch.Tensor,
                               n_steps: int, ess_threshold: float, n_bisect: int, rho: float,
                               n_jitter: int, max_temper: int, workspace: torch.Tensor,
                               gtol: float = LBFGS_GTOL, max_iter: int = LBFGS_MAX_ITER,
                               mem: int = LBFGS_MEM, max_back: int = LBFGS_MAX_BACK,
                               ckpt_every: int = 8) -> dict:
    """sch_pf_nudged_cycle with the Matern-type noise; dLambdac [n][n_steps][nx]."""
    mc, tc, oc = model.c(), mt.c(), obs.c()
    n = m.shape[0]
    _state(model, n, m=m, u=u)
    _inc(n, n_steps, model.nx, dLambdac=dLambdac)
    _ws(workspace, nudged_workspace_bytes_matern(model, n, n_steps, n_jitter, ckpt_every))
    st = SchCycleStats()
    opts = SchLbfgsOpts(gtol, max_iter, mem, max_back)
    _check(lib().sch_pf_nudged_cycle_matern(C.byref(mc), C.byref(tc), C.byref(oc), seed, cycle,
                                            m.shape[0], n_steps, ess_threshold, n_bisect, rho,
                                            n_jitter, max_temper, C.byref(opts), ckpt_every,
                                            _dev(m, name="m"), _dev(u, name="u"),
                                            _dev(dLambdac, name="dLambdac"),
                                            _dev(workspace, torch.uint8, "workspace"),
                                            C.byref(st), _stream()))
    return st.as_dict()


@dataclass
class Instance:
    """One filter of a batch: its grid, state and observations (GPU tensors)."""
    xi: torch.Tensor     # [n_modes][nx]
    m: torch.Tensor      # [n][nx] in/out
    u: torch.Tensor      # [n][nx] in/out
    logw: torch.Tensor   # [n] in/out
    y: torch.Tensor      # [cycles][n_obs]
    sigma: torch.Tensor  # [n_obs]
    seed: int
    threads: int = 0

    def c(self) -> SchInstanceC:
        return SchInstanceC(int(self.m.shape[1]), int(self.m.shape[0]), _dev(self.xi, name="xi"),
                            _dev(self.m, name="m"), _dev(self.u, name="u"),
                            _dev(self.logw, name="logw"), _dev(self.y, name="y"),
                            _dev(self.sigma, name="sigma"), self.seed, self.threads)


class Batch:
    """Handle of sch_batch_*: many bootstrap filters advanced together.  Keeps
    the instance tensors and the workspace alive until close()."""

    def __init__(self, L: float, alpha: float, mu: float, dt: float, n_modes: int, n_steps: int,
                 n_obs: int, ess_frac: float, instances: list[Instance],
                 picard_tol: float = 1e-13, picard_max: int = 50):
        self.instances = list(instances)
        self.params = SchBatchParamsC(L, alpha, mu, dt, n_modes, n_steps, n_obs, ess_frac,
                                      picard_tol, picard_max)
        arr = (SchInstanceC * len(self.instances))(*[i.c() for i in self.instances])
        self._arr = arr
        nb = int(lib().sch_batch_workspace_bytes(C.byref(self.params), len(arr), arr))
        if nb <= 0:
            raise SchError(SCH_E_ARG, lib().sch_last_error().decode())
        self.workspace = torch.empty(nb, dtype=torch.uint8, device=self.instances[0].m.device)
        h = _vp()
        _check(lib().sch_batch_create(C.byref(self.params), len(arr), arr,
                                      _dev(self.workspace, torch.uint8, "workspace"), nb,
                                      C.byref(h), _stream()))
        self.handle = h

    def run(self, cycle0: int, n_cycles: int = 1, use_graph: bool = False):
        _check(lib().sch_batch_run(self.handle, cycle0, n_cycles, 1 if use_graph else 0,
                                   _stream()))

    def read(self) -> dict:
        k = len(self.instances)
        ess = (C.c_double * k)()
        res = (C.c_int32 * k)()
        st = (C.c_int32 * k)()
        it = C.c_int64(0)
        _check(lib().sch_batch_read(self.handle, ess, res, st, C.byref(it), _stream()))
        return {"ess": list(ess), "resampled": list(res), "status": list(st),
                "picard_iters": it.value}

    def close(self):
        if getattr(self, "handle", None):
            lib().sch_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------- warm-start network
def sch_mlp_param_count(n_in: int, n_hidden: int, n_out: int) -> int:
    return int(lib().sch_mlp_param_count(n_in, n_hidden, n_out))


@dataclass
class Mlp:
    """Warm-start network: float32 master parameters and their bfloat16 weight
    copy (GPU tensors, sizes checked against the layer widths)."""
    n_in: int
    n_hidden: int
    n_out: int
    params: torch.Tensor        # float32 [sch_mlp_param_count]
    weights_bf16: torch.Tensor  # bfloat16 [H F + H H + O H]

    def c(self) -> SchMlpC:
        _at_least(self.params, sch_mlp_param_count(self.n_in, self.n_hidden, self.n_out),
                  "params")
        _at_least(self.weights_bf16, self.n_hidden * self.n_in + self.n_hidden * self.n_hidden
                  + self.n_out * self.n_hidden, "weights_bf16")
        return SchMlpC(self.n_in, self.n_hidden, self.n_out,
                       _dev(self.params, torch.float32, "params"),
                       _dev(self.weights_bf16, torch.bfloat16, "weights_bf16"))


def sch_mlp_workspace_bytes(net: Mlp, batch: int) -> int:
    nc = net.c()
    return int(lib().sch_mlp_workspace_bytes(C.byref(nc), batch))


def sch_mlp_sync(net: Mlp):
    nc = net.c()
    _check(lib().sch_mlp_sync(C.byref(nc), _stream()))


def sch_mlp_forward(net: Mlp, X: torch.Tensor, Y: torch.Tensor, workspace: torch.Tensor):
    nc = net.c()
    B = X.shape[0]
    _shape(X, (B, net.n_in), "X")
    _shape(Y, (B, net.n_out), "Y")
    _ws(workspace, sch_mlp_workspace_bytes(net, B))
    _check(lib().sch_mlp_forward(C.byref(nc), X.shape[0], _dev(X, torch.bfloat16, "X"),
                                 _dev(Y, torch.float32, "Y"),
                                 _dev(workspace, torch.uint8, "workspace"), _stream()))


def sch_mlp_backward(net: Mlp, X: torch.Tensor, Y: torch.Tensor, T: torch.Tensor,
                     loss: torch.Tensor, grad: torch.Tensor, workspace: torch.Tensor):
    nc = net.c()
    B = X.shape[0]
    _shape(X, (B, net.n_in), "X")
    _shape(Y, (B, net.n_out), "Y")
    _shape(T, (B, net.n_out), "T")
    _at_least(loss, 1, "loss")
    _at_least(grad, net.params.numel(), "grad")
    _ws(workspace, sch_mlp_workspace_bytes(net, B))
    _check(lib().sch_mlp_backward(C.byref(nc), X.shape[0], _dev(X, torch.bfloat16, "X"),
                                  _dev(Y, torch.float32, "Y"), _dev(T, torch.float32, "T"),
                                  _dev(loss, torch.float64, "loss"),
                                  _dev(grad, torch.float32, "grad"),
                                  _dev(workspace, torch.uint8, "workspace"), _stream()))


def sch_mlp_adam(net: Mlp, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int,
                 lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    nc = net.c()
    k = net.params.numel()
    _at_least(grad, k, "grad")
    _at_least(m, k, "m")
    _at_least(v, k, "v")
    _check(lib().sch_mlp_adam(C.byref(nc), _dev(grad, torch.float32, "grad"),
                              _dev(m, torch.float32, "m"), _dev(v, torch.float32, "v"), step,
                              lr, beta1, beta2, eps, _stream()))


def sch_mlp_features(model: Model, obs: Obs, u: torch.Tensor, mean: torch.Tensor | None,
                     sdev: torch.Tensor | None, X: torch.Tensor | None = None,
                     raw: torch.Tensor | None = None, misfit: torch.Tensor | None = None):
    mc, oc = model.c(), obs.c()
    _check(lib().sch_mlp_features(C.byref(mc), C.byref(oc), u.shape[0], _dev(u, name="u"),
                                  _dev(mean, torch.float32, "mean"),
                                  _dev(sdev, torch.float32, "sdev"),
                                  _dev(X, torch.bfloat16, "X"), _dev(raw, torch.float32, "raw"),
                                  _dev(misfit, name="misfit"), _stream()))


def sch_mlp_colstats(A: torch.Tensor, mean: torch.Tensor, sdev: torch.Tensor):
    _check(lib().sch_mlp_colstats(A.shape[0], A.shape[1], _dev(A, torch.float32, "A"),
                                  _dev(mean, torch.float32, "mean"),
                                  _dev(sdev, torch.float32, "sdev"), _stream()))


def sch_mlp_encode(raw: torch.Tensor, mean: torch.Tensor, sdev: torch.Tensor, X: torch.Tensor):
    _check(lib().sch_mlp_encode(raw.shape[0], raw.shape[1], _dev(raw, torch.float32, "raw"),
                                _dev(mean, torch.float32, "mean"),
                                _dev(sdev, torch.float32, "sdev"),
                                _dev(X, torch.bfloat16, "X"), _stream()))


def sch_mlp_targets(dLam: torch.Tensor, mean: torch.Tensor | None, sdev: torch.Tensor | None,
                    T: torch.Tensor):
    n = dLam.shape[0]
    cols = dLam.numel() // n
    _check(lib().sch_mlp_targets(n, cols, _dev(dLam, name="dLambda"),
                                 _dev(mean, torch.float32, "mean"),
                                 _dev(sdev, torch.float32, "sdev"),
                                 _dev(T, torch.float32, "T"), _stream()))


def sch_mlp_controls(Y: torch.Tensor, mean: torch.Tensor, sdev: torch.Tensor,
                     misfit: torch.Tensor | None, threshold: float, dLam: torch.Tensor,
                     mode: torch.Tensor | None = None, keep_mode: int = 0):
    n = Y.shape[0]
    cols = Y.numel() // n
    _at_least(dLam, n * cols, "dLambda")
    _vec(n, misfit=misfit, mode=mode)
    _check(lib().sch_mlp_controls(n, cols, _dev(Y, torch.float32, "Y"),
                                  _dev(mean, torch.float32, "mean"),
                                  _dev(sdev, torch.float32, "sdev"),
                                  _dev(misfit, name="misfit"), threshold,
                                  _dev(dLam, name="dLambda"), _dev(mode, torch.int32, "mode"),
                                  keep_mode, _stream()))


TIMING_KINDS = ("window", "jitter", "temper", "resample", "gather", "other", "nudge", "adjoint")


def sch_timing_enable(on: bool = True):
    _check(lib().sch_timing_enable(1 if on else 0))


def sch_timing_reset():
    _check(lib().sch_timing_reset())


def sch_timing_read() -> dict:
    k = len(TIMING_KINDS)
    ms = (C.c_double * k)()
    la = (C.c_int64 * k)()
    it = (C.c_int64 * k)()
    _check(lib().sch_timing_read(ms, la, it))
    return {name: {"ms": ms[i], "launches": la[i], "iters": it[i]}
            for i, name in enumerate(TIMING_KINDS)}


TUNE_THREADS = 2


def sch_tune_set(key: int, value: int):
    _check(lib().sch_tune_set(key, value))


def sch_tune_get(key: int) -> int:
    return int(lib().sch_tune_get(key))
