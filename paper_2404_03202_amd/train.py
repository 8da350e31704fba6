"""Training loop of Alg. 1 on the C ABI: render, photometric loss (Eq. 17:
L1 and, with lambda_dssim > 0, the SSIM term), backward,
densification statistics and the Adam step every iteration; densify and
prune every `densify_interval` iterations up to `densify_until`, opacity
reset every `reset_interval`.  Every step runs in the library's kernels;
this module only holds the tensors and the schedule.

Hyperparameters are 3DGS's published defaults (the paper's supplement with
its own values is not available); the densification threshold applies to
||dL/ds||, s the uniform ERP screen coordinate of Eq. 4.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import omnigs as B


@dataclasses.dataclass
class TrainSettings:
    extent: float = 1.0
    lr_means_init: float = 1.6e-4
    lr_means_final: float = 1.6e-6
    lr_steps: int = 30000
    lr_sh_dc: float = 2.5e-3
    lr_sh_rest: float = 2.5e-3 / 20.0
    lr_logits: float = 0.05
    lr_log_scales: float = 5e-3
    lr_quats: float = 1e-3
    densify_from: int = 500
    densify_until: int = 15000
    densify_interval: int = 100
    reset_interval: int = 3000
    grad_threshold: float = 2e-4
    percent_dense: float = 0.01
    min_opacity: float = 0.005
    max_screen: float = 20.0
    big_fraction: float = 0.1
    split_shrink: float = 1.6
    reset_value: float = 0.01
    lambda_dssim: float = 0.2  # weight of the SSIM term of Eq. 17 (0: L1 only)


def logit(p):
    p = np.clip(np.asarray(p, np.float64), 1e-7, 1 - 1e-7)
    return np.log(p / (1.0 - p))


class Trainer:
    """Holds the raw parameters, the Adam moments, the statistics and the
    activated copies the rasterizer reads.

    capacity_slack (None: every forward reads its instance counts back): the
    forwards take instance and block-entry capacities of capacity_slack times
    the largest counts read so far and read nothing back.  An iteration whose
    forward overflowed leaves the parameters, moments and statistics as they
    were (its overflow flag gates the Adam and statistics kernels on the
    device); the flags are read `lag` iterations later, and such an iteration
    is then run again with its counts read back, which regrows the
    capacities."""

    def __init__(self, gaussians: dict, settings: TrainSettings | None = None, device="cuda:0", seed=0,
                 render_settings: dict | None = None, capacity_slack: float | None = None, lag: int = 2):
        self.s = settings or TrainSettings()
        self.device = device
        self.render_settings = render_settings
        self.slack = capacity_slack
        self.lag = lag
        self.cap = None      # (instances, block entries) once counted
        self._pending = []   # (overflow flag, camera, target, mask) of recent capacity-mode iterations
        self.redone = 0
        g = gaussians
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        self.p = dict(means=f(g["means"]), log_scales=f(np.log(g["scales"])), quats=f(g["quats"]),
                      logits=f(logit(g["opacities"])), sh=f(g["sh"]), sh_degree=int(g["sh_degree"]))
        self._fresh_state()
        self.step_count = 0
        self.rng = np.random.default_rng(seed)

    def _fresh_state(self):
        z = lambda t: torch.zeros_like(t)
        self.m1 = {k: (z(v) if torch.is_tensor(v) else v) for k, v in self.p.items()}
        self.m2 = {k: (z(v) if torch.is_tensor(v) else v) for k, v in self.p.items()}
        n = self.n
        self.stats = dict(accum=torch.zeros(n, device=self.device), denom=torch.zeros(n, device=self.device),
                          max_radius=torch.zeros(n, device=self.device))
        self._activate()

    @property
    def n(self):
        return int(self.p["means"].shape[0])

    def _activate(self):
        self.act = dict(means=self.p["means"], scales=torch.exp(self.p["log_scales"]).contiguous(),
                        quats=self.p["quats"], opacities=torch.sigmoid(self.p["logits"]).contiguous(), sh=self.p["sh"],
                        sh_degree=self.p["sh_degree"])

    def lrs(self):
        t = min(self.step_count / self.s.lr_steps, 1.0)
        lr_m = self.s.extent * float(np.exp(np.log(self.s.lr_means_init) * (1 - t) + np.log(self.s.lr_means_final) * t))
        return dict(means=lr_m, sh_dc=self.s.lr_sh_dc, sh_rest=self.s.lr_sh_rest, logits=self.s.lr_logits,
                    log_scales=self.s.lr_log_scales, quats=self.s.lr_quats)

    def step(self, camera: dict, target: torch.Tensor, mask: torch.Tensor | None = None):
        """One iteration; returns the loss tensor (device).  ``mask`` [H, W]:
        per-pixel loss weights (a camera's "rows" skips bottom rows
        outright)."""
        self.step_count += 1
        loss = self._iterate(camera, target, mask, self.cap if self.slack else None)
        self._settle(self.lag)
        j, s = self.step_count, self.s
        if j <= s.densify_until:
            if j >= s.densify_from and j % s.densify_interval == 0:
                self.densify(screen=j > s.reset_interval)
            if j % s.reset_interval == 0:
                B.omnigs_reset_opacity(self.p, self.m1, self.m2, s.reset_value)
                self.act["opacities"] = torch.sigmoid(self.p["logits"]).contiguous()
        return loss

    def _iterate(self, camera, target, mask, cap):
        fwd = B.omnigs_forward(self.act, camera, self.render_settings, capacity=cap)
        if self.s.lambda_dssim > 0.0 or mask is not None:
            loss, dl = B.omnigs_photometric_loss(fwd.image, target, self.s.lambda_dssim, mask=mask)
        else:
            loss, dl = B.omnigs_l1_loss(fwd.image, target)
        grads = B.omnigs_backward(self.act, camera, self.render_settings, fwd, dl)
        B.omnigs_accumulate_stats(fwd, grads, self.stats, skip=fwd.overflow)
        # the activated copies are rewritten in place by the Adam kernel
        B.omnigs_adam_step(self.p, grads, self.m1, self.m2, self.lrs(), self.step_count, self.act,
                           skip=fwd.overflow)
        if cap is not None:
            self._pending.append((fwd.overflow, camera, target, mask))
        elif self.slack:
            want = (int(self.slack * fwd.n_instances) + 1, int(self.slack * fwd.n_entries) + 1)
            self.cap = want if self.cap is None else (max(self.cap[0], want[0]), max(self.cap[1], want[1]))
        return loss

    def _settle(self, keep: int):
        """Read the overflow flags of all but the last `keep` capacity-mode
        iterations; run the overflowed ones again with their counts read back."""
        while len(self._pending) > keep:
            overflow, camera, target, mask = self._pending.pop(0)
            if int(overflow.item()):
                self.redone += 1
                self._iterate(camera, target, mask, None)

    def flush(self):
        """Settle every pending capacity-mode iteration."""
        self._settle(0)

    def densify(self, screen: bool = True):
        self.flush()
        n_before = self.n
        s = self.s
        noise = torch.from_numpy(self.rng.standard_normal((self.n, 2, 3)).astype(np.float32)).to(self.device)
        settings = dict(grad_threshold=s.grad_threshold, percent_dense=s.percent_dense, extent=s.extent,
                        min_opacity=s.min_opacity, max_screen=s.max_screen if screen else 0.0,
                        big_fraction=s.big_fraction, split_shrink=s.split_shrink)
        self.p, self.m1, self.m2, self.stats = B.omnigs_densify(self.p, self.m1, self.m2, self.stats, noise, settings)
        self._activate()
        if self.cap is not None and self.n > n_before:  # more Gaussians: scale the capacities with them
            f = self.n / max(n_before, 1)
            self.cap = (int(self.cap[0] * f) + 1, int(self.cap[1] * f) + 1)
