"""Pin for the oracle's likelihood-ratio tangents (differentiation form): the
derivative of a smooth observable of the density with respect to
theta = (H, w, x0), estimated by the tangents, must agree with central finite
differences under common random numbers (same seed on both sides of theta),
averaged over independent seeds, within 4.5 standard errors.

gamma0 is held fixed at 0.45, so only the kick density and the pair acceptance
depend on theta.  The packet starts next to the barrier so that the derivative
is far from zero at T = 3 (30 steps, annihilation every 10).

Mode 2 replaces the x0 score -2q cot(2q(x - x0)) by derivative ghost pairs
(the x0-derivative of the pair intensity, -2q c cos, realised as ghosts with
tangents -/+2q s created with probability c|cos|)."""
import numpy as np
import pytest

import workloads as W

THETA0 = (0.3, 1.0, 0.0)


def _phi(O, seed, theta, mode=1):
    cfg = W.gaussian_barrier_small(N0=np.array([2000]), gamma0=0.45, track_tangent=mode, seed=seed)
    cfg["init"] = dict(cfg["init"], mean_x=[-4.0, 0.0])
    cfg = W.with_theta(cfg, H=theta[0], width=theta[1], center=theta[2])
    s = O.OracleSim(cfg)
    s.run(30, 10)
    x = -60 + 0.25 + 0.5 * np.arange(240)
    g = 0.5 * (1 + np.tanh(x / 2.0))
    return float(g @ s.density()[0]), s.density_tangent()[0] @ g


def test_tangent_matches_crn_finite_differences(oracle_mod):
    """Both tangent modes against the same finite differences.  Mode 2 (x0 by
    derivative ghost pairs) must also agree, carry the same (H, w) tangents
    bit for bit (its ghosts hold zero there and add nothing to the sums), and
    estimate the x0 derivative with a clearly smaller spread than the
    likelihood-ratio score, whose second moment diverges."""
    R, h = 300, 0.02
    fd = np.zeros((R, 3))
    lr = np.zeros((R, 3))
    wd = np.zeros((R, 3))
    for r in range(R):
        p1, lr[r] = _phi(oracle_mod, 5000 + r, THETA0, 1)
        p2, wd[r] = _phi(oracle_mod, 5000 + r, THETA0, 2)
        assert p1 == p2          # the tangent mode never changes the particles
        for c in range(3):
            tp, tm = list(THETA0), list(THETA0)
            tp[c] += h
            tm[c] -= h
            fd[r, c] = (_phi(oracle_mod, 5000 + r, tp)[0] - _phi(oracle_mod, 5000 + r, tm)[0]) / (2 * h)
    for est in (lr, wd):
        d = fd - est
        se = d.std(0, ddof=1) / np.sqrt(R)
        assert np.all(np.abs(d.mean(0)) < 4.5 * se), (fd.mean(0), est.mean(0), se)
    # the H derivative is large and sharply estimated: a dropped or wrong score shows
    assert abs(lr[:, 0].mean()) > 10 * lr[:, 0].std() / np.sqrt(R)
    assert np.array_equal(lr[:, :2], wd[:, :2])
    # x0 by derivative pairs: far from zero (a sign error fails the agreement
    # above) and with at most a third of the score's variance here
    assert abs(wd[:, 2].mean()) > 10 * wd[:, 2].std() / np.sqrt(R)
    assert wd[:, 2].var() < lr[:, 2].var() / 3.0
