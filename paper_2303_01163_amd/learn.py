"""Training of the learned correction (include/asdsm_learn.h) on pairs that ASDSM itself generates.

A training pair is (r_k, implied correction A^{-1} r_k) for an iterate u_k of a plain ASDSM run
(Algorithm 4): the network sees the residual window with the coarse-plane positions and the cell
Peclet numbers, and the residual loss mean (rhat - A' c)^2 measures its proposal c against the
exact correction in the A^T A norm without ever forming A^{-1} r_k.  Problems are the seeded
``sinbump3d`` family (alpha_i log-uniform in [0.1, 1], beta_i uniform in [-5, 5], sinusoid-product
plus Gaussian-bump solutions): several coefficient draws, several sources per draw, one plain run
per source, and a few random windows of the fine residual per iterate.

Every step runs in the HIP library: the plain solves (asdsm_solve, one refinement step per call),
the residuals (asdsm_residual), the network input (asdsm_net_features), forward and backward passes
(asdsm_net_gradient) and the Adam updates (asdsm_net_adam).  This module only orchestrates them.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import asdsm
from .workloads import make_problem

__all__ = ["TrainConfig", "train_correction", "problem_tensors", "discrete_manufactured"]


class TrainConfig:
    """Schedule of a training run: ``plans`` coefficient draws x ``sources`` right-hand sides x
    ``iters`` plain refinement steps x ``windows`` residual windows per iterate = pairs."""

    def __init__(self, level=7, coarse_level=0, plans=8, sources=10, iters=32, windows=4, lr=1e-3,
                 lr_final=5e-5, seed=1000, log_every=512, loss_every=8):
        self.level = int(level)
        self.coarse_level = int(coarse_level)
        self.plans = int(plans)
        self.sources = int(sources)
        self.iters = int(iters)
        self.windows = int(windows)
        self.lr = float(lr)
        self.lr_final = float(lr_final)
        self.seed = int(seed)
        self.log_every = int(log_every)
        self.loss_every = int(loss_every)   # the loss is read back (a host sync) every loss_every pairs

    @property
    def pairs(self) -> int:
        return self.plans * self.sources * self.iters * self.windows


def problem_tensors(P, device):
    import torch
    s = torch.from_numpy(P.s_flat()).to(device)
    g = torch.from_numpy(P.g_flat()).to(device)
    return s, g


def discrete_manufactured(plan, P, device):
    """(s, g, u): the source that makes the manufactured grid function u of problem P the exact
    solution of the discrete system (b_ff = A_ff u), so that the algebraic error of an iterate is
    measured against u itself.  s = -(b_ff(s = 0) - A_ff u) = A_ff u - (Dirichlet terms), from the
    library's own residual."""
    import torch
    g = torch.from_numpy(P.g_flat()).to(device)
    u = torch.from_numpy(np.ascontiguousarray(P.u_exact.reshape(-1, order="F"))).to(device)
    zero = torch.zeros_like(u)
    r0, _ = plan.residual(u, zero, g)
    return -r0, g, u


def _lr(cfg: TrainConfig, step: int, total: int) -> float:
    """Cosine decay from lr to lr_final over the run."""
    c = 0.5 * (1.0 + math.cos(math.pi * min(step, total) / max(total, 1)))
    return cfg.lr_final + (cfg.lr - cfg.lr_final) * c


def train_correction(net: "asdsm.Net", cfg: TrainConfig, log=None) -> dict:
    """Train ``net`` (built for windows of n^3 voxels, n <= N_f) in place; returns a summary with the
    loss history (mean of the sampled losses -- every ``loss_every``-th pair -- over each block of
    ``log_every`` pairs)."""
    import torch
    rng = np.random.default_rng(cfg.seed)
    total = cfg.pairs
    step = 0
    first_loss = None
    losses = []
    block = []
    t0 = time.perf_counter()
    solve_ms = 0.0
    n = net.n
    for ip in range(cfg.plans):
        coef_seed = cfg.seed + 7919 * ip
        C = make_problem("sinbump3d", cfg.level, seed=coef_seed)
        plan = asdsm.Plan(3, C.alpha, C.beta, cfg.level, cfg.coarse_level, seed=coef_seed,
                          device=net.device.index, stream=net.stream)
        net.bind(plan)
        nf = plan.n_f
        if n > nf:
            raise ValueError(f"network volume {n} exceeds the fine mesh {nf}")
        u = torch.empty(plan.n_fine, dtype=torch.float64, device=net.device)
        for js in range(cfg.sources):
            P = make_problem("sinbump3d", cfg.level, seed=coef_seed + 1 + js, alpha=C.alpha, beta=C.beta)
            s, g = problem_tensors(P, net.device)
            ts = time.perf_counter()
            plan.solve(s, g, u=u, max_iter=0)                       # u^(0), Algorithm 1
            solve_ms += 1e3 * (time.perf_counter() - ts)
            for k in range(cfg.iters):
                r, rn = plan.residual(u, s, g)                     # r and ||r||_2
                for _ in range(cfg.windows):
                    off = rng.integers(0, nf - n + 1, size=3)
                    x, rhat = net.features(r, rn * rn, off)
                    sample = step % cfg.loss_every == 0
                    loss, _ = net.gradient(x, rhat, loss="residual", want_grad=False, want_loss=sample)
                    net.adam(_lr(cfg, step, total))
                    if step == 0:
                        first_loss = loss
                    step += 1
                    if sample:
                        block.append(loss)
                    if step % cfg.log_every == 0 and block:
                        losses.append(float(np.mean(block)))
                        block = []
                        if log:
                            log(f"pairs {step}/{total} loss {losses[-1]:.4f} "
                                f"{time.perf_counter() - t0:.1f} s")
                ts = time.perf_counter()
                plan.solve(s, g, u=u, max_iter=1, rtol=0.0, stag_window=0, resume=True, k0=k)
                solve_ms += 1e3 * (time.perf_counter() - ts)
        plan.close()
    if block:
        losses.append(float(np.mean(block)))
    net.plan = None
    torch.cuda.synchronize(net.device)
    return {"pairs": step, "first_loss": first_loss, "loss_hist": losses, "seconds": time.perf_counter() - t0,
            "solve_seconds": solve_ms / 1e3, "config": vars(cfg).copy()}
