"""Pins for the sp2 resampling steps of the oracle.

- Alg. 2 (residual bootstrap): copies_i = floor(n w~_i) + multinomial(N_r, r_i/R).
  For tiny inputs the exact law of the copy vector is enumerated here and
  compared by chi-square with the oracle's draws; E[copies_i] = n A_i / S; the
  copy total is n (class counts preserved).
- Lemma 1: the bootstrap's mean-square error of <phi, .> is below 4 ||phi||^2/n.
- Rounding step of Alg. 3: E[n_nu] = m_nu and Var = f(1-f) with f the
  fractional part; 128-bit cell values give the exact integer part.
"""
import itertools
import math

import numpy as np
from scipy import stats


def exact_law(A):
    n = len(A)
    S = sum(A)
    k = [n * a // S for a in A]
    r = [n * a - ki * S for a, ki in zip(A, k)]
    Nr = n - sum(k)
    R = S * Nr
    law = {}
    for combo in itertools.product(range(n), repeat=Nr):
        c = list(k)
        for i in combo:
            c[i] += 1
        p = 1.0
        for i in combo:
            p *= r[i] / R
        law[tuple(c)] = law.get(tuple(c), 0.0) + p
    return law


def test_residual_bootstrap_exact_law(oracle_mod):
    A = [3, 5, 1, 7, 2]
    law = exact_law(A)
    draws = 30000
    counts = {}
    for step in range(draws):
        c = tuple(int(v) for v in oracle_mod.bootstrap_class(A, seed=11, step=step))
        assert sum(c) == len(A)
        counts[c] = counts.get(c, 0) + 1
    assert set(counts) <= set(law)
    obs = np.array([counts.get(c, 0) for c in law])
    exp = np.array([law[c] * draws for c in law])
    keep = exp > 5
    chi2 = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-3


def test_bootstrap_mean_and_lemma1(oracle_mod):
    rng = np.random.default_rng(5)
    n = 64
    w = rng.uniform(0.01, 1.0, n)
    A = np.floor(w * 2.0 ** 32).astype(np.uint64)
    S = int(A.sum())
    phi = np.cos(np.arange(n))                       # ||phi|| <= 1
    target = float((phi * (n * A.astype(np.float64) / S)).sum() / n)
    reps = 4000
    C = np.array([oracle_mod.bootstrap_class(A, seed=3, step=s) for s in range(reps)])
    assert np.all(C.sum(1) == n)
    mean = C.mean(0)
    expect = n * A.astype(np.float64) / S
    sd = np.sqrt(np.maximum(C.var(0), 1e-12) / reps)
    assert np.all(np.abs(mean - expect) < 5 * sd + 1e-9)
    mse = np.mean(((C * phi).sum(1) / n - target) ** 2)
    assert mse <= 4.0 / n


def test_bootstrap_degenerate_classes(oracle_mod):
    assert list(oracle_mod.bootstrap_class([], step=0)) == []
    assert list(oracle_mod.bootstrap_class([0, 0, 0])) == [0, 0, 0]
    # equal weights: every particle is kept exactly once, no draws
    assert list(oracle_mod.bootstrap_class([2**32] * 7)) == [1] * 7


def test_rounding_mean_and_variance(oracle_mod):
    num, den = 7, 3
    v = np.array([oracle_mod.round_cell(num, den, cell=c) for c in range(40000)])
    f = 1.0 / 3.0
    assert set(np.unique(v)) == {2, 3}
    assert abs(v.mean() - 7 / 3) < 5 * math.sqrt(f * (1 - f) / len(v))
    assert abs(v.var() - f * (1 - f)) < 0.01


def test_rounding_wide_integers(oracle_mod):
    import random
    rng = random.Random(9)
    for _ in range(200):
        den = rng.randrange(1, 2**62) << rng.randrange(0, 26)
        num = den * rng.randrange(0, 2**40) + rng.randrange(0, den)
        got = oracle_mod.round_cell(num, den, cell=rng.randrange(0, 2**40))
        assert got in (num // den, num // den + 1)
    # exact multiples never round up
    assert oracle_mod.round_cell(12 << 90, 3 << 90) == 4
