"""Pins for the sp2 cell values of the oracle (Sec. 4.3).

After the residual bootstrap of each sign class (Alg. 2), the histogram of
Eq. boostrap_histogram gives cell nu the signed mass
N_alpha (lambda+ n~+_nu / N+ + lambda- n~-_nu / N-) with
lambda+- = (1/N_alpha) sum of the class's weights (Eq. lambda), which Alg. 3's
rounding step turns into an integer count.  The weights enter once, quantised
to A = floor(|w| 2^32) (the oracle's one reading of the floating sums).

- Exact: on hand-built two-class ensembles with N+ != N-, every cell's count
  is floor or ceil of that mass, evaluated here with exact fractions from the
  weights and the oracle's per-cell bootstrap counts, and carries its sign;
  the bootstrap keeps each class's size; the regenerated particles follow the
  counts.
- Mass: over many seeds the mean signed count of a cell equals the summed
  (quantised) weight of the cell, the expectation both resampling steps keep.
- Physics: the sp2 density at T = 20 matches split-step Schroedinger, as the
  sp1 one does.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W

Q32 = 1 << 32


def _grid_cfg(seed=0, strategy="sp2"):
    cfg = W.gaussian_barrier_small(N0=np.array([1]), strategy=strategy, seed=seed)
    cfg["grid"] = {"x_lo": -4.0, "x_hi": 4.0, "nx": 8, "k_lo": -2.0, "k_hi": 2.0, "nk": 4}
    return cfg


def _cells(cfg, x, k):
    g = cfg["grid"]
    qx = (x - g["x_lo"]) / ((g["x_hi"] - g["x_lo"]) / g["nx"])
    qk = (k - g["k_lo"]) / ((g["k_hi"] - g["k_lo"]) / g["nk"])
    ok = (qx >= 0) & (qx < g["nx"]) & (qk >= 0) & (qk < g["nk"])
    return np.where(ok, qx.astype(np.int64) + g["nx"] * qk.astype(np.int64), -1)


def _ensemble(rng, n_plus=37, n_minus=11):
    """Particles spread over a few cells of the 8 x 4 grid (and two outside),
    weights of both signs that are not multiples of 2^-32."""
    n = n_plus + n_minus
    x = rng.uniform(-4.5, 4.5, n)          # some outside [-4, 4)
    x[:6] = rng.uniform(-1.0, 0.0, 6)      # a shared cell
    k = rng.uniform(-1.9, 1.9, n)
    k[:6] = 0.3
    w = np.concatenate([rng.uniform(0.05, 1.7, n_plus), -rng.uniform(0.05, 2.3, n_minus)])
    perm = rng.permutation(n)
    return x[perm], k[perm], w[perm]


def _quant(w):
    return math.floor(abs(Fraction(float(w))) * Q32)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_sp2_cell_counts_are_the_rounded_bootstrap_histogram(oracle_mod, seed):
    rng = np.random.default_rng(100 + seed)
    x, k, w = _ensemble(rng, n_plus=37 + seed, n_minus=11 + 3 * seed)
    cfg = _grid_cfg(seed=seed)
    s = oracle_mod.OracleSim(cfg)
    s.set_particles(0, x[None, :], k[None, :], w=w, ids=np.arange(len(w), dtype=np.uint64))
    s.keep_cells()
    s.annihilate()
    nplus, nminus, cnt = s.cells()

    nu = _cells(cfg, x, k)
    inside = nu >= 0
    pos, neg = inside & (w > 0), inside & (w < 0)
    Np, Nm = int(pos.sum()), int(neg.sum())
    assert Np != Nm and Np > 0 and Nm > 0
    Sp = sum(_quant(v) for v in w[pos])
    Sm = sum(_quant(v) for v in w[neg])
    # Alg. 2 keeps the class sizes, and a class's copies stay in its cells
    assert nplus.sum() == Np and nminus.sum() == Nm
    assert np.all(nplus[np.setdiff1d(np.arange(len(nplus)), nu[pos])] == 0)
    assert np.all(nminus[np.setdiff1d(np.arange(len(nminus)), nu[neg])] == 0)
    nonint = 0
    for c in range(len(cnt)):
        # N_alpha (lambda+ n+/N+ + lambda- n-/N-), lambda+- N_alpha = +-S+-/2^32
        m = Fraction(Sp, Q32) * Fraction(int(nplus[c]), Np) - Fraction(Sm, Q32) * Fraction(int(nminus[c]), Nm)
        lo, hi = math.floor(abs(m)), math.ceil(abs(m))
        assert abs(int(cnt[c])) in (lo, hi), (c, m, cnt[c])
        if cnt[c] != 0:
            assert np.sign(cnt[c]) == (1 if m > 0 else -1), (c, m, cnt[c])
        nonint += lo != hi
    assert nonint >= 3   # the rounding step is exercised
    # regenerated ensemble: |n_nu| particles of weight sgn(n_nu) in cell nu
    p = s.particles()
    nu2 = _cells(cfg, p["x"][0], p["k"][0])
    assert np.array_equal(np.bincount(nu2, minlength=len(cnt)), np.abs(cnt))
    assert np.array_equal(p["w"], np.sign(cnt[nu2]).astype(np.float64))


def test_sp2_mean_signed_count_equals_cell_weight(oracle_mod):
    rng = np.random.default_rng(7)
    x, k, w = _ensemble(rng, n_plus=23, n_minus=9)
    nu = _cells(_grid_cfg(), x, k)
    ncell = 32
    target = np.zeros(ncell)
    for c, v in zip(nu, w):
        if c >= 0:
            target[c] += math.copysign(_quant(v), v) / Q32
    R = 3000
    acc = np.zeros((R, ncell))
    for r in range(R):
        s = oracle_mod.OracleSim(_grid_cfg(seed=r))
        s.set_particles(0, x[None, :], k[None, :], w=w, ids=np.arange(len(w), dtype=np.uint64))
        s.keep_cells()
        s.annihilate()
        acc[r] = s.cells()[2]
    mean = acc.mean(0)
    se = acc.std(0, ddof=1) / np.sqrt(R)
    occupied = target != 0
    assert occupied.sum() >= 8
    z = (mean - target)[occupied] / np.maximum(se[occupied], 1e-12)
    assert np.all(np.abs(z) < 4.5), (mean[occupied], target[occupied], z)
    # and the total is the net weight in the box
    tot = acc.sum(1)
    assert abs(tot.mean() - target.sum()) < 4.5 * tot.std(ddof=1) / np.sqrt(R) + 1e-9


def _schroedinger_density(T, H=0.3, w=1.0, x0=0.0, L=400.0, n=16384, dts=0.005):
    x = -L / 2 + np.arange(n) * L / n
    psi = (2 * np.pi) ** -0.25 * np.exp(-(x + 15) ** 2 / 4 + 1.5j * x)
    V = H * np.exp(-(x - x0) ** 2 / (2 * w * w))
    k = 2 * np.pi * np.fft.fftfreq(n, d=L / n)
    half = np.exp(-0.5j * V * dts)
    kin = np.exp(-0.5j * k * k * dts)
    for _ in range(int(round(T / dts))):
        psi = half * np.fft.ifft(kin * np.fft.fft(half * psi))
    return x, np.abs(psi) ** 2


def test_sp2_density_matches_schroedinger(oracle_mod):
    """The whole sp2 path (wp pairs, bootstrap, cell values, rounding): the
    transmitted probability and the coarse density at T = 20 agree with
    split-step Schroedinger.  Swapping N+ and N- in the cell value, or the
    classes' lambdas, moves the transmission by far more than the bound."""
    x, rho = _schroedinger_density(20.0)
    dx = x[1] - x[0]
    cfg = W.gaussian_barrier_small(N0=np.array([100_000]), seed=2, strategy="sp2")
    s = oracle_mod.OracleSim(cfg)
    s.run(200, 10)
    d = s.density()[0]
    centres = -60 + 0.25 + 0.5 * np.arange(240)
    P_wbrw = d[centres > 0].sum() * 0.5
    P_exact = rho[x > 0].sum() * dx
    assert abs(P_wbrw - P_exact) < 0.01, (P_wbrw, P_exact)
    coarse = d.reshape(24, 10).sum(1) * 0.5
    exact = np.array([rho[(x >= lo) & (x < lo + 5)].sum() * dx for lo in np.arange(-60, 60, 5)])
    assert np.abs(coarse - exact).sum() < 0.06, np.abs(coarse - exact).sum()
