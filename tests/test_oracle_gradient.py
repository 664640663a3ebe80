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


def _phi_sp2(O, seed, theta, steps, every, N, mean_x):
    cfg = W.gaussian_barrier_small(N0=np.array([N]), gamma0=0.45, track_tangent=1, seed=seed,
                                   strategy="sp2")
    cfg["init"] = dict(cfg["init"], mean_x=[mean_x, 0.0])
    cfg = W.with_theta(cfg, H=theta[0], width=theta[1], center=theta[2])
    s = O.OracleSim(cfg)
    s.run(steps, every)
    x = -60 + 0.25 + 0.5 * np.arange(240)
    g = 0.5 * (1 + np.tanh(x / 2.0))
    return float(g @ s.density()[0]), s.density_tangent()[0] @ g


def test_sp2_tangent_is_the_pathwise_derivative(oracle_mod):
    """sp2 without annihilation: the weights are smooth in (H, x0) for fixed
    random numbers, and the H and x0 tangents are their exact derivatives, so
    each seed's tangent equals its own central difference (h = 1e-4) to the
    difference's truncation error.  The width tangent uses the kick density's
    score while the difference moves the kicks (q scales as 1/w), so those two
    agree in the mean only."""
    R, h = 300, 1e-4
    tg = np.zeros((R, 3))
    fd = np.zeros((R, 3))
    for r in range(R):
        _, tg[r] = _phi_sp2(oracle_mod, 7000 + r, THETA0, 15, 0, 500, -2.0)
        for c in range(3):
            tp, tm = list(THETA0), list(THETA0)
            tp[c] += h
            tm[c] -= h
            fd[r, c] = (_phi_sp2(oracle_mod, 7000 + r, tp, 15, 0, 500, -2.0)[0]
                        - _phi_sp2(oracle_mod, 7000 + r, tm, 15, 0, 500, -2.0)[0]) / (2 * h)
    # A seed where some kick's sine changes sign within +-h swaps that pair's
    # children (and with them their ids and later draws): a jump of the size of
    # the vanishing pair weight.  Such seeds are rare; the rest match closely.
    for c in (0, 2):
        scale = np.max(np.abs(tg[:, c]))
        assert scale > 0.01
        err = np.abs(tg[:, c] - fd[:, c]) / scale
        assert np.median(err) < 1e-6 and np.mean(err < 1e-5) >= 0.98, (c, np.sort(err)[-5:])
    d = tg[:, 1] - fd[:, 1]
    assert abs(d.mean()) < 4.5 * d.std(ddof=1) / np.sqrt(R)


def test_sp2_tangent_mean_equals_sp1(oracle_mod):
    """With annihilation every 10 steps, sp1 and sp2 estimate the same
    expected density (both annihilations preserve the expected signed mass per
    cell and place it uniformly), so their tangents estimate the same
    derivative: the means over independent seeds agree within 4.5 standard
    errors, on a case where the derivative is far from zero."""
    R = 300
    a = np.array([_phi(oracle_mod, 5000 + r, THETA0, 2)[1] for r in range(R)])
    b = np.array([_phi_sp2(oracle_mod, 9000 + r, THETA0, 30, 10, 2000, -4.0)[1] for r in range(R)])
    se = np.sqrt(a.var(0, ddof=1) / R + b.var(0, ddof=1) / R)
    assert np.all(np.abs(a.mean(0) - b.mean(0)) < 4.5 * se), (a.mean(0), b.mean(0), se)
    assert np.all(np.abs(b.mean(0)) > 10 * b.std(0, ddof=1) / np.sqrt(R))


def test_tangent_sums_are_exact_fixed_point_sums(oracle_mod):
    """Cell and bin sums of tangents are exact sums of trunc(D 2^32) (32.32
    fixed point), read back as floor(Q / 2^32) + (Q mod 2^32) 2^-32: checked
    here with Python integers on the oracle's own per-particle tangents, for
    the tangent density and the backward contraction, and against the
    floating sums within the truncation bound n 2^-32 per bin."""
    from fractions import Fraction
    import math
    cfg = W.gaussian_barrier_small(N0=np.array([3000]), gamma0=0.45, track_tangent=1, seed=3)
    s = oracle_mod.OracleSim(cfg)
    s.run(25, 10)
    assert s.stats()["range_errors"] == 0
    nb, lo, hi = 60, -30.0, 30.0
    dx = (hi - lo) / nb
    parts = [s.particles(), s.particles(ghost=True)]
    Q = np.zeros((3, nb), dtype=object)
    Q[:] = 0
    fl = np.zeros((3, nb))
    cnt = np.zeros(nb, dtype=np.int64)
    for p in parts:
        q = (p["x"][0] - lo) / dx
        for i in np.flatnonzero((q >= 0) & (q < nb)):
            j = int(q[i])
            cnt[j] += 1
            for c in range(3):
                D = float(p["D"][i, c])
                Q[c, j] += math.trunc(Fraction(D) * 2**32)
                fl[c, j] += D
    val = np.array([[float(Q[c, j] // 2**32) + float(Q[c, j] % 2**32) * 2.0**-32 for j in range(nb)]
                    for c in range(3)])
    denom = 3000 * dx
    J = s.density_tangent(nbins=nb, lo=lo, hi=hi)[0]
    assert np.array_equal(J, val / denom)
    assert np.all(np.abs(val - fl) <= cnt * 2.0**-32 + 1e-12 * np.abs(fl) + 1e-300)
    g = np.sin(np.arange(nb) * 0.3)
    got = s.density_vjp(g, nbins=nb, lo=lo, hi=hi)[0]
    for c in range(3):
        acc = 0.0
        for j in range(nb):
            acc = acc + g[j] * val[c, j]
        assert got[c] == acc / denom
