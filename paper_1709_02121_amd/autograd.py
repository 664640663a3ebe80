"""torch.autograd.Function for the position density at time T of one
Gaussian-barrier instance, differentiable in theta = (H, w, x0).

Forward: runs the walk with per-particle tangents carried forward (kernels of
libwbrw.so): likelihood-ratio scores of the kick density and of the pair
acceptance (track_tangent 1), the same for (H, w) with the x0 derivative
carried by derivative ghost pairs of finite variance (track_tangent 2), or,
for sp2, pathwise weight derivatives.  It returns the density.  Backward: the
library's vector-Jacobian kernel contracts the upstream gradient with the
tangents of every particle and ghost at T.  Because the tangents are carried
forward, the backward pass needs no replay of the forward one: checkpoints
(ensemble snapshots every `snapshot_every` steps) are restart points for the
caller, handed over in `checkpoints` if given, never kept by the graph.  The
auxiliary rate gamma0 is held fixed, so the jump times carry no score.
"""
from __future__ import annotations

import copy

import numpy as np
import torch

from . import Simulation


def theta_config(cfg, theta):
    """Copy of a one-instance, one-Gaussian-component workload with
    (H, w, x0) = theta and tangent tracking on (the workload's mode, 1 if it
    has none; sp2 takes mode 1)."""
    c = copy.deepcopy(cfg)
    if int(c["B"]) != 1 or len(c["components"]) != 1 or c["components"][0]["kind"] != "gauss":
        raise ValueError("the density gradient needs one instance with one Gaussian component")
    if not float(c["gamma0"]) > 0:
        raise ValueError("gamma0 must be fixed (> 0) so that it does not depend on theta")
    th = [float(v) for v in theta]
    comp = c["components"][0]
    comp["H"] = np.array([th[0]])
    comp["width"] = np.array([th[1]])
    comp["center"] = np.array([th[2]])
    mode = int(c.get("track_tangent", 0)) or 1
    if c["strategy"] == "sp2" and mode != 1:
        raise ValueError("sp2 carries pathwise tangents (track_tangent 1) only")
    c["track_tangent"] = mode
    return c


class WBRWDensity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, cfg, steps, annihilate_every, snapshot_every, device, checkpoints):
        sim = Simulation(theta_config(cfg, theta.detach().cpu().numpy()), device=device)
        for s in range(int(steps)):
            sim.step(1)
            if annihilate_every and (s + 1) % annihilate_every == 0:
                sim.annihilate()
            if checkpoints is not None and snapshot_every and (s + 1) % snapshot_every == 0:
                checkpoints.append((s + 1, sim.snapshot()))
        rho = sim.density()[0]
        ctx.sim = sim
        ctx.theta_dtype = theta.dtype
        ctx.theta_device = theta.device
        return rho

    @staticmethod
    def backward(ctx, grad_rho):
        grad = ctx.sim.density_vjp(grad_rho.reshape(1, -1))[0]
        grad = grad.to(device=ctx.theta_device, dtype=ctx.theta_dtype)
        ctx.sim = None
        return grad, None, None, None, None, None, None


def density(theta, cfg, steps=None, annihilate_every=None, snapshot_every=None, device="cuda:0",
            checkpoints=None):
    """rho(x, T; theta) on the workload's density bins; differentiable in theta.
    checkpoints: a list that receives (step, snapshot) every snapshot_every
    steps (restart points for wbrw_restore), or None for no checkpoints."""
    steps = cfg["steps"] if steps is None else steps
    every = cfg.get("annihilate_every", 0) if annihilate_every is None else annihilate_every
    snap = cfg.get("snapshot_every", 0) if snapshot_every is None else snapshot_every
    return WBRWDensity.apply(theta, cfg, steps, every, snap, device, checkpoints)
