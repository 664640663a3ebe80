"""Pins for the oracle's series-based log, sin and cos.

Each is compared with a 50-digit mpmath evaluation; the error must stay within
3 units in the last place for log (the rounding of (m-1)/(m+1) costs up to about
2.3 ulp) and 2 for sin/cos, over the ranges the method uses (log of (0,1], sines
of kernel phases up to a few thousand radians, Box-Muller angles) and beyond.
A wrong coefficient, a missing series term or a wrong reduction constant gives
errors of many ulp.
"""
import mpmath
import numpy as np

mpmath.mp.dps = 50


def _ulp_err(got, f, xs):
    worst = 0.0
    for g, x in zip(got, xs):
        ref = f(mpmath.mpf(float(x)))
        r = float(ref)
        if r == 0.0:
            assert g == 0.0
            continue
        ulp = np.spacing(abs(r))
        worst = max(worst, float(abs(mpmath.mpf(float(g)) - ref) / ulp))
    return worst


def test_dlog_ulp(oracle_mod):
    rng = np.random.default_rng(1)
    xs = np.concatenate([
        1.0 - rng.random(3000),                    # arguments 1-u of the life-length draw
        np.exp(rng.uniform(-700, 700, 1500)),      # wide range
        1.0 + rng.uniform(-1e-3, 1e-3, 500),       # near 1
        [2.0 ** -53, 0.5, 1.0, 2.0, np.sqrt(0.5), np.nextafter(np.sqrt(0.5), 0)],
    ])
    got = oracle_mod.dlog(xs)
    assert got[-4] == 0.0  # log(1) is exactly 0
    assert _ulp_err(got, mpmath.log, xs) <= 3.0


def test_dsin_dcos_ulp(oracle_mod):
    rng = np.random.default_rng(2)
    xs = np.concatenate([
        rng.uniform(0, 2 * np.pi, 1500),           # Box-Muller angles
        rng.uniform(-4000, 4000, 1500),            # kernel phases 2q(x - x0)
        rng.uniform(-1e-6, 1e-6, 300),
        rng.uniform(-1e5, 1e5, 300),
        np.pi / 4 * np.arange(-16, 17),
    ])
    for fo, fm in ((oracle_mod.dsin, mpmath.sin), (oracle_mod.dcos, mpmath.cos)):
        got = fo(xs)
        # relative ulp error except where the true value is tiny (near zeros of
        # sin/cos the absolute error is bounded by the reduction's accuracy)
        rel = []
        for g, x in zip(got, xs):
            ref = fm(mpmath.mpf(float(x)))
            r = float(ref)
            if abs(r) < 1e-3:
                assert abs(g - r) < 1e-19 + 4e-16 * abs(x) * 1e-16 + 2e-19
                continue
            rel.append(float(abs(mpmath.mpf(float(g)) - ref) / np.spacing(abs(r))))
        assert max(rel) <= 2.0


def test_sin_cos_pythagoras_and_symmetry(oracle_mod):
    rng = np.random.default_rng(3)
    xs = rng.uniform(-50, 50, 2000)
    s, c = oracle_mod.dsin(xs), oracle_mod.dcos(xs)
    assert np.max(np.abs(s * s + c * c - 1.0)) < 1e-15
    assert np.array_equal(oracle_mod.dsin(-xs), -s)
    assert np.array_equal(oracle_mod.dcos(-xs), c)
