"""Seeded synthetic workloads for the signed-particle Wigner branching random walk.

This module only describes inputs: physical parameters, grids, initial-state
parameters, per-instance parameter draws and the tabulated Fourier transform of
the soft-Coulomb potential.  It performs none of the method's arithmetic, and it
is the only code shared by the oracle's tests and the HIP path's tests and
benchmark.

The paper measures on no public dataset; its test problems are a Gaussian
barrier scattering in 2D phase space and a Helium-like system in 4D phase space
(Sec. 5).  The workloads below re-parameterise those problems with hbar = m = 1.
"""
from __future__ import annotations

import copy
import math

import numpy as np

KIND = {"gauss": 0, "table": 1}
STRATEGY = {"sp1": 0, "sp2": 1}


def _gauss_component(B, H, width, center):
    return {
        "kind": "gauss",
        "axis": 0,
        "H": np.broadcast_to(np.asarray(H, dtype=np.float64), (B,)).copy(),
        "width": np.broadcast_to(np.asarray(width, dtype=np.float64), (B,)).copy(),
        "center": np.broadcast_to(np.asarray(center, dtype=np.float64), (B,)).copy(),
    }


def gaussian_barrier_small(**over):
    """Gaussian barrier V(x) = 0.3 exp(-x^2/2), f0 = (1/pi) exp(-(x+15)^2/2 - 2(k-1.5)^2)
    sampled as 1e4 signed particles; dt = 0.1 x 100 steps, annihilation every 10
    steps on a 240 x 128 grid over x in [-60,60), k in [-8,8); seed 0."""
    cfg = {
        "name": "gaussian_barrier_1e4",
        "dim": 1,
        "strategy": "sp1",
        "B": 1,
        "instance_offset": 0,
        "seed": 0,
        "hbar": 1.0,
        "mass": 1.0,
        "dt": 0.1,
        "gamma0": 0.0,          # <= 0: derived as gamma_scale * xi_hat / 2
        "gamma_scale": 1.0,
        "components": [_gauss_component(1, 0.3, 1.0, 0.0)],
        "N0": np.array([10_000], dtype=np.int64),
        "init": {"mean_x": [-15.0, 0.0], "sigma_x": [1.0, 1.0],
                 "mean_k": [1.5, 0.0], "sigma_k": [0.5, 0.5]},
        "grid": {"x_lo": -60.0, "x_hi": 60.0, "nx": 240,
                 "k_lo": -8.0, "k_hi": 8.0, "nk": 128},
        "steps": 100,
        "annihilate_every": 10,
        "density": {"axis": 0, "nbins": 240, "lo": -60.0, "hi": 60.0},
        "capacity_factor": 8.0,
        "track_tangent": 0,
    }
    return _override(cfg, over)


def gaussian_barrier_large(strategy="sp1", **over):
    """Same barrier at 1e7 initial particles (capacity 2e8), 1000 steps,
    annihilation every 10 steps on a 2000 x 512 grid over x in [-200,200),
    k in [-8,8); run as sp1 (pair generation) or sp2 (bootstrap filter)."""
    cfg = gaussian_barrier_small()
    cfg.update({
        "name": f"gaussian_barrier_1e7_{strategy}",
        "strategy": strategy,
        "N0": np.array([10_000_000], dtype=np.int64),
        "grid": {"x_lo": -200.0, "x_hi": 200.0, "nx": 2000,
                 "k_lo": -8.0, "k_hi": 8.0, "nk": 512},
        "steps": 1000,
        "density": {"axis": 0, "nbins": 2000, "lo": -200.0, "hi": 200.0},
        "capacity": 200_000_000,
    })
    return _override(cfg, over)


def soft_coulomb_table(n=4096, q_lo=-8.0, q_hi=8.0, strength=1.0):
    """|F[v](2 q_j)| at bin midpoints q_j for v(r) = strength / sqrt(r^2 + 1),
    whose transform is F[v](s) = 2 strength K0(|s|)."""
    from scipy.special import k0

    dq = (q_hi - q_lo) / n
    q = q_lo + (np.arange(n) + 0.5) * dq
    return 2.0 * abs(strength) * k0(np.abs(2.0 * q))


def helium_soft_coulomb(**over):
    """Helium-like 4D phase space (x1,x2,k1,k2) with
    V = -2/sqrt(x1^2+1) - 2/sqrt(x2^2+1) + 1/sqrt((x1-x2)^2+1): three kernel
    components (nucleus-electron 1, nucleus-electron 2, electron-electron) with
    kicks (1,0), (0,1), (1,-1); tabulated transform on 4096 points over
    q in [-8,8); f0 a product of Gaussians (sigma_x = 1, sigma_k = 1/2) centred at
    x = -2 and +2, k = 0, sampled as 1e7 particles; 100^4 cells over
    x in [-10,10)^2, k in [-4,4)^2; dt = 0.05 x 400 steps."""
    ne = soft_coulomb_table(strength=2.0)
    ee = soft_coulomb_table(strength=1.0)
    tab = lambda t, axis, sgn: {"kind": "table", "axis": axis, "table": t,
                                "q_lo": -8.0, "q_hi": 8.0, "sgn": sgn, "center": 0.0}
    cfg = {
        "name": "helium_soft_coulomb_1e7",
        "dim": 2,
        "strategy": "sp1",
        "B": 1,
        "instance_offset": 0,
        "seed": 0,
        "hbar": 1.0,
        "mass": 1.0,
        "dt": 0.05,
        "gamma0": 0.0,
        "gamma_scale": 1.0,
        "components": [tab(ne, 0, -1.0), tab(ne, 1, -1.0), tab(ee, 2, 1.0)],
        "N0": np.array([10_000_000], dtype=np.int64),
        "init": {"mean_x": [-2.0, 2.0], "sigma_x": [1.0, 1.0],
                 "mean_k": [0.0, 0.0], "sigma_k": [0.5, 0.5]},
        "grid": {"x_lo": -10.0, "x_hi": 10.0, "nx": 100,
                 "k_lo": -4.0, "k_hi": 4.0, "nk": 100},
        "steps": 400,
        "annihilate_every": 10,
        "density": {"axis": 0, "nbins": 200, "lo": -10.0, "hi": 10.0},
        "capacity_factor": 40.0,
        "track_tangent": 0,
    }
    return _override(cfg, over)


def batched_barriers(B=256, seed=0, **over):
    """B independent Gaussian-barrier instances: numpy default_rng(seed) draws,
    in order, H_b ~ U[0.1,0.5], w_b ~ U[0.5,2], log10 N_b ~ U[4,6]; gamma0_b = H_b
    (gamma_scale 1); 500 steps, annihilation every 10 on a 240 x 128 grid each.
    Capacity 16 N_b per instance: the smallest instances (N_b near 1e4 on 30720
    cells, fewer particles than cells) keep growing between resamplings and
    reach 9.5 N_b within the 500 steps."""
    rng = np.random.default_rng(seed)
    H = rng.uniform(0.1, 0.5, size=B)
    w = rng.uniform(0.5, 2.0, size=B)
    N = np.rint(10.0 ** rng.uniform(4.0, 6.0, size=B)).astype(np.int64)
    cfg = gaussian_barrier_small()
    cfg.update({
        "name": f"batched_barriers_{B}",
        "B": B,
        "components": [{"kind": "gauss", "axis": 0, "H": H, "width": w,
                        "center": np.zeros(B)}],
        "N0": N,
        "steps": 500,
        "capacity_factor": 16.0,
    })
    return _override(cfg, over)


def differentiation(**over):
    """Gaussian barrier at 1e7 particles, 500 steps, sp1, annihilation every 10,
    theta0 = (H, w, x0) = (0.3, 1, 0), gamma0 fixed at 0.45 (1.5 xi_hat/2), density
    on 2000 bins over [-200,200), snapshots every 50 steps."""
    cfg = gaussian_barrier_large("sp1")
    cfg.update({
        "name": "differentiation_1e7",
        "steps": 500,
        "gamma0": 0.45,
        "track_tangent": 1,
        "snapshot_every": 50,
        "fd_h": 1e-3,
    })
    return _override(cfg, over)


def time_dependent_barriers(**over):
    """Double barrier whose left barrier switches (Sec. 5.6): heights
    0.8 (0.5 + 0.5 cos(pi + 0.1 t)) at x = -10 and 0.8 at x = +10, both of
    width 2 (exp(-(x -+ 10)^2/8)); packet from x = -15 (k = 1.5, sigma_x = 1),
    gamma0 = 1, dt = 0.1, 600 steps, annihilation every 10 on 240 x 128 over
    [-60,60) x [-8,8).  The switching barrier is placed on the left, as the
    paper's description of the dynamics has it."""
    cfg = gaussian_barrier_small()
    comp_a = _gauss_component(1, 0.8, 2.0, -10.0)
    comp_a["modulation"] = {"a": 0.5, "b": 0.5, "omega": 0.1, "phase": math.pi}
    comp_b = _gauss_component(1, 0.8, 2.0, 10.0)
    cfg.update({
        "name": "time_dependent_barriers_1e4",
        "components": [comp_a, comp_b],
        "gamma0": 1.0,
        "steps": 600,
    })
    return _override(cfg, over)


def cat_state_wigner(x, k, sep=10.0, center=-15.0, k0=1.5, sigma=1.0):
    """Wigner function (hbar = 1, integral 1) of the normalised superposition of
    two Gaussian packets of width sigma at center -+ sep/2 with wave number k0;
    its interference term makes it negative on fringes of period 2 pi / sep in k."""
    a, b = center - sep / 2, center + sep / 2
    g = lambda c: np.exp(-(x - c) ** 2 / (2 * sigma ** 2) - 2 * sigma ** 2 * (k - k0) ** 2) / np.pi
    overlap = np.exp(-sep ** 2 / (8 * sigma ** 2))
    cross = 2.0 * np.exp(-(x - center) ** 2 / (2 * sigma ** 2) - 2 * sigma ** 2 * (k - k0) ** 2) \
        * np.cos(sep * (k - k0)) / np.pi
    return (g(a) + g(b) + cross) / (2.0 * (1.0 + overlap))


def cat_state_barrier(N0=200_000, **over):
    """Signed initial data: the cat state above tabulated at the centres of a
    240 x 512 grid over [-60,60) x [-8,8) (dk = 1/32 resolves the fringes of
    period 0.63) and sampled by importance sampling from the histogram (Alg. 3);
    Gaussian barrier 0.3 exp(-x^2/2); dt = 0.1."""
    cfg = gaussian_barrier_small(N0=np.array([N0]))
    cfg["grid"] = dict(cfg["grid"], nk=512)
    g = cfg["grid"]
    dx = (g["x_hi"] - g["x_lo"]) / g["nx"]
    dk = (g["k_hi"] - g["k_lo"]) / g["nk"]
    xc = g["x_lo"] + (np.arange(g["nx"]) + 0.5) * dx
    kc = g["k_lo"] + (np.arange(g["nk"]) + 0.5) * dk
    hist = cat_state_wigner(xc[None, :], kc[:, None])      # [nk][nx]: cell nu = ix + nx ik
    cfg.update({"name": "cat_state_barrier", "init_histogram": hist.reshape(1, -1),
                "capacity_factor": 12.0})
    return _override(cfg, over)


def with_theta(cfg, H=None, width=None, center=None):
    """Copy of a single-Gaussian workload with barrier parameters replaced."""
    c = copy.deepcopy(cfg)
    comp = c["components"][0]
    if H is not None:
        comp["H"] = np.full(c["B"], float(H))
    if width is not None:
        comp["width"] = np.full(c["B"], float(width))
    if center is not None:
        comp["center"] = np.full(c["B"], float(center))
    return c


def scaled(cfg, N0=None, steps=None, **over):
    """Copy of a workload at another size (for parity runs the oracle finishes)."""
    c = copy.deepcopy(cfg)
    if N0 is not None:
        c["N0"] = np.broadcast_to(np.asarray(N0, dtype=np.int64), (c["B"],)).copy()
    if steps is not None:
        c["steps"] = int(steps)
    return _override(c, over)


def _override(cfg, over):
    for k, v in over.items():
        cfg[k] = v
    return cfg


ALL = {
    "gaussian_barrier_1e4": gaussian_barrier_small,
    "gaussian_barrier_1e7_sp1": lambda: gaussian_barrier_large("sp1"),
    "gaussian_barrier_1e7_sp2": lambda: gaussian_barrier_large("sp2"),
    "helium_soft_coulomb_1e7": helium_soft_coulomb,
    "batched_barriers_256": batched_barriers,
    "differentiation_1e7": differentiation,
    "time_dependent_barriers_1e4": time_dependent_barriers,
    "cat_state_barrier": cat_state_barrier,
}
