"""Learned warm start of the nudging stages (an extension of section 3.1.3).

A perceptron maps a particle's window-start features (observation misfit
y - P u and the velocity u, standardised) to the controls dLambda of the
window, learned from the solutions of plain nudging; its prediction seeds the
L-BFGS stages of ``sch_nudge_run``.  Particles whose misfit norm exceeds the
99th percentile of the training misfits keep the plain start (zero), so plain
nudging is both the fallback and, through its own convergence test, the arbiter
of the prediction.

Orchestration only: features, standardisation statistics, the network's
forward and backward passes, Adam and the conversion to controls all run in
the library's kernels (``sch_mlp_*``); this module allocates tensors, picks
minibatches and calls them in order.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import sch
from . import workloads as W


@dataclass
class Dataset:
    """Training pairs gathered from plain nudging."""
    raw: torch.Tensor      # float32 [N][F] unscaled features
    misfit: torch.Tensor   # float64 [N]
    dLam: torch.Tensor     # float64 [N][S][Q] plain-nudging controls


class WarmStart:
    def __init__(self, n_obs: int, nx: int, n_steps: int, n_modes: int, hidden: int = 256,
                 seed: int = W.MASTER_SEED, device: str = "cuda"):
        self.n_obs, self.nx, self.n_steps, self.n_modes = n_obs, nx, n_steps, n_modes
        self.F, self.H, self.O = n_obs + nx, hidden, n_steps * n_modes
        p = W.mlp_init_params(self.F, self.H, self.O, seed)
        assert p.size == sch.sch_mlp_param_count(self.F, self.H, self.O)
        nw = self.H * self.F + self.H * self.H + self.O * self.H
        self.net = sch.Mlp(self.F, self.H, self.O,
                           torch.tensor(p, dtype=torch.float32, device=device),
                           torch.empty(nw, dtype=torch.bfloat16, device=device))
        sch.sch_mlp_sync(self.net)
        self.m = torch.zeros_like(self.net.params)
        self.v = torch.zeros_like(self.net.params)
        self.grad = torch.zeros_like(self.net.params)
        self.step = 0
        self.device = device
        self.x_mean = self.x_sdev = self.y_mean = self.y_sdev = None
        self.threshold = float("inf")

    # ----------------------------------------------------------------- data
    def collect(self, model: sch.Model, obs: sch.Obs, m: torch.Tensor, u: torch.Tensor,
                dW: torch.Tensor, ws: torch.Tensor | None = None) -> Dataset:
        """Plain nudging of one window from (m, u) with the revealed increments
        dW; returns the window-start features and the controls found (m, u
        advance to the nudged window end)."""
        n = u.shape[0]
        raw = torch.empty((n, self.F), dtype=torch.float32, device=self.device)
        mis = torch.empty(n, dtype=torch.float64, device=self.device)
        sch.sch_mlp_features(model, obs, u, None, None, None, raw, mis)
        dLam = torch.zeros_like(dW)
        logG = torch.empty(n, dtype=torch.float64, device=self.device)
        sch.sch_nudge_run(model, obs, m, u, dW, dLam, logG, workspace=ws)
        return Dataset(raw, mis, dLam)

    def fit_scaling(self, data: Dataset):
        """Feature / target standardisation and the fallback threshold from the
        training set."""
        N = data.raw.shape[0]
        self.x_mean = torch.empty(self.F, dtype=torch.float32, device=self.device)
        self.x_sdev = torch.empty_like(self.x_mean)
        sch.sch_mlp_colstats(data.raw, self.x_mean, self.x_sdev)
        t = torch.empty((N, self.O), dtype=torch.float32, device=self.device)
        sch.sch_mlp_targets(data.dLam, None, None, t)
        self.y_mean = torch.empty(self.O, dtype=torch.float32, device=self.device)
        self.y_sdev = torch.empty_like(self.y_mean)
        sch.sch_mlp_colstats(t, self.y_mean, self.y_sdev)
        self.threshold = float(np.quantile(data.misfit.cpu().numpy(), 0.99))

    def encode(self, data: Dataset):
        """bfloat16 network inputs and float32 targets of a dataset."""
        N = data.raw.shape[0]
        X = torch.empty((N, self.F), dtype=torch.bfloat16, device=self.device)
        sch.sch_mlp_encode(data.raw, self.x_mean, self.x_sdev, X)
        T = torch.empty((N, self.O), dtype=torch.float32, device=self.device)
        sch.sch_mlp_targets(data.dLam, self.y_mean, self.y_sdev, T)
        return X, T

    # ----------------------------------------------------------------- training
    def train(self, X: torch.Tensor, T: torch.Tensor, epochs: int, batch: int = 256,
              lr: float = 1e-3, seed: int = 0, log=None) -> list[float]:
        """Adam on minibatches of contiguous rows in a shuffled order of
        batches; returns the mean loss of every epoch."""
        N = X.shape[0]
        ws = torch.empty(sch.sch_mlp_workspace_bytes(self.net, batch), dtype=torch.uint8,
                         device=self.device)
        Y = torch.empty((batch, self.O), dtype=torch.float32, device=self.device)
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        starts = np.arange(0, N - batch + 1, batch)
        g = np.random.default_rng(seed)
        history = []
        for ep in range(epochs):
            acc = torch.zeros(1, dtype=torch.float64, device=self.device)
            for s0 in g.permutation(starts):
                xb, tb = X[s0:s0 + batch], T[s0:s0 + batch]
                sch.sch_mlp_forward(self.net, xb, Y, ws)
                sch.sch_mlp_backward(self.net, xb, Y, tb, loss, self.grad, ws)
                self.step += 1
                sch.sch_mlp_adam(self.net, self.grad, self.m, self.v, self.step, lr)
                acc += loss
            history.append(float(acc.item()) / len(starts))
            if log:
                log(f"epoch {ep}: loss {history[-1]:.4f}")
        return history

    # ----------------------------------------------------------------- inference
    def predict(self, model: sch.Model, obs: sch.Obs, u: torch.Tensor, dLam: torch.Tensor,
                fallback: bool = True, mode: torch.Tensor | None = None,
                keep_mode: int = sch.NUDGE_KEEP) -> torch.Tensor:
        """Warm-start controls for the particles u into dLam [n][S][Q]; returns
        the misfit norms.  mode (int32 [n], optional) receives the start mode
        of every particle for sch_pf_nudged_cycle_warm: keep_mode where the
        prediction is used, NUDGE_FROM_ZERO (plain nudging) where the misfit is
        above the training range."""
        n = u.shape[0]
        X = torch.empty((n, self.F), dtype=torch.bfloat16, device=self.device)
        mis = torch.empty(n, dtype=torch.float64, device=self.device)
        sch.sch_mlp_features(model, obs, u, self.x_mean, self.x_sdev, X, None, mis)
        Y = torch.empty((n, self.O), dtype=torch.float32, device=self.device)
        ws = torch.empty(sch.sch_mlp_workspace_bytes(self.net, n), dtype=torch.uint8,
                         device=self.device)
        sch.sch_mlp_forward(self.net, X, Y, ws)
        sch.sch_mlp_controls(Y, self.y_mean, self.y_sdev, mis if fallback else None,
                             self.threshold, dLam, mode, keep_mode)
        return mis

    def nudged_cycle(self, model: sch.Model, obs: sch.Obs, seed: int, cycle: int,
                     m: torch.Tensor, u: torch.Tensor, dLam: torch.Tensor, n_steps: int,
                     ess_threshold: float, n_bisect: int, rho: float, n_jitter: int,
                     max_temper: int, workspace: torch.Tensor, keep_mode: int = sch.NUDGE_KEEP,
                     **lbfgs) -> dict:
        """One cycle of the nudged filter with the network's controls: every
        particle whose misfit lies in the training range takes the predicted
        controls (as they are with NUDGE_KEEP, as the L-BFGS start with
        NUDGE_FROM_GIVEN), the others are nudged from zero; then tempering and
        jittering with the weights W~ as in sch_pf_nudged_cycle."""
        mode = torch.empty(u.shape[0], dtype=torch.int32, device=self.device)
        self.predict(model, obs, u, dLam, True, mode, keep_mode)
        return sch.sch_pf_nudged_cycle_warm(model, obs, seed, cycle, m, u, dLam, mode, n_steps,
                                            ess_threshold, n_bisect, rho, n_jitter, max_temper,
                                            workspace, **lbfgs)


def concat(parts: list[Dataset]) -> Dataset:
    return Dataset(torch.cat([p.raw for p in parts]), torch.cat([p.misfit for p in parts]),
                   torch.cat([p.dLam for p in parts]))
