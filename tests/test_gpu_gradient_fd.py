"""The differentiation workload at full size on the GPU: the tangent gradient
of a smooth functional of the density against central finite differences
with common random numbers.

1e7 particles, 500 steps (annihilation every 10, gamma0 fixed at 0.45),
density on 2000 bins over [-200, 200); the functional is <g, rho> with a
smooth g.  For each of R = 32 seeds the tangent run gives d<g, rho>/d theta
(x0 by derivative ghost pairs, whose variance is finite; H and w by
likelihood-ratio scores, the same as mode 1's), and runs at theta +- h e_j,
h = 1e-3, under the same seed give the central difference.  Both estimate
the same derivative, so their difference over seeds has mean zero: checked
within 4 standard errors per parameter, with the H estimate itself far from
zero (so the check has power).
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.timeout(900)
def test_tangent_gradient_matches_crn_finite_differences_1e7():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1709_02121_amd as P
    base = W.differentiation(track_tangent=2, capacity=60_000_000)
    steps, every, h, R = 500, 10, 1e-3, 32
    nb = base["density"]["nbins"]
    x = -200 + (np.arange(nb) + 0.5) * (400.0 / nb)
    g = np.tanh(x / 25.0)
    gt = torch.tensor(g, dtype=torch.float64, device="cuda").reshape(1, nb)
    theta0 = np.array([0.3, 1.0, 0.0])
    lr = np.zeros((R, 3))
    fd = np.zeros((R, 3))

    def functional(cfg):
        sim = P.Simulation(cfg)
        sim.run(steps, every, use_graph=True)
        v = float((sim.density()[0] * gt[0]).sum())
        sim.close()
        del sim
        return v

    for s in range(R):
        cfg = dict(base, seed=s)
        sim = P.Simulation(cfg)
        sim.run(steps, every, use_graph=True)
        lr[s] = sim.density_vjp(gt)[0].cpu().numpy()
        sim.close()
        del sim
        plain = dict(cfg, track_tangent=0)
        for j in range(3):
            th_p, th_m = theta0.copy(), theta0.copy()
            th_p[j] += h
            th_m[j] -= h
            fp = functional(W.with_theta(plain, H=th_p[0], width=th_p[1], center=th_p[2]))
            fm = functional(W.with_theta(plain, H=th_m[0], width=th_m[1], center=th_m[2]))
            fd[s, j] = (fp - fm) / (2 * h)
        if s % 8 == 7:
            say(f"fd check: {s + 1} seeds; LR mean {lr[:s + 1].mean(0)}, FD mean {fd[:s + 1].mean(0)}")
    d = fd - lr
    se = d.std(0, ddof=1) / np.sqrt(R)
    say(f"LR {lr.mean(0)} +- {lr.std(0, ddof=1) / np.sqrt(R)}; FD {fd.mean(0)} +- "
        f"{fd.std(0, ddof=1) / np.sqrt(R)}; FD - LR {d.mean(0)} +- {se}")
    assert np.all(np.abs(d.mean(0)) < 4 * se), (d.mean(0), se)
    lr_se = lr.std(0, ddof=1) / np.sqrt(R)
    assert abs(lr.mean(0)[0]) > 6 * lr_se[0], (lr.mean(0), lr_se)
