"""GPU parity at the benchmark sizes, in the launch configuration bench.py
times (default persistent grids and plain launches; the batched form with the
autotuner and graph replay).  The oracle computes every particle of these
ensembles in tens of seconds, so the comparison is over the whole ensemble,
bit for bit, not over a sample: the 1e7-particle Gaussian barrier in sp1 and
sp2, the differentiation form in every tangent mode (sp1 scores, sp1
derivative pairs, sp2 pathwise), and the 1e7-particle 4D
helium model.  The batched form (256 instances, 5.5e7 particles) is compared
on sampled instances, each replayed by the oracle on its own through the
instance key offset."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1709_02121_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as O
    O.build()
    return O


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def same(a, b, what, fields=("x", "k", "sign", "w", "id")):
    for f in fields:
        if f not in a or f not in b:
            continue
        x, y = np.asarray(a[f]), np.asarray(b[f])
        assert x.shape == y.shape, (what, f, x.shape, y.shape)
        bad = np.flatnonzero(x != y) if x.ndim == 1 else np.flatnonzero((x != y).any(axis=0))
        assert bad.size == 0, f"{what}: {f} differs at {bad[:5]} of {x.shape}"


def stats_equal(g, r, what, b=0, rb=None):
    sg, so = g.stats(b), r.stats(b if rb is None else rb)
    keys = ["n", "events", "pairs", "killed", "escaped", "max_depth", "event_cap_hits"]
    if g.cfg["strategy"] == "sp2":
        keys += ["S_plus", "S_minus", "N_plus", "N_minus"]
    for k in keys:
        assert sg[k] == so[k], (what, b, k, sg[k], so[k])


def exact(a, b, what):
    """Tangents: bit-identical (cell and bin sums are exact fixed-point sums)."""
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    if np.array_equal(a, b):
        return
    bad = np.flatnonzero(a.ravel() != b.ravel())
    rel = np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))
    raise AssertionError(f"{what}: {len(bad)} elements differ, first at {bad[:5]} (max rel {rel:.3e})")


def epoch_parity(P, O, cfg, steps, what, tangents=False):
    """Init, `steps` steps (compared before annihilation), one annihilation
    (compared), and the density readout, on the whole ensemble."""
    say(f"{what}: init N0={int(cfg['N0'][0])}")
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    same(g.particles(), r.particles(), f"{what} init")
    g.step(steps)
    r.step(steps)
    say(f"{what}: {steps} steps n={r.count()}")
    stats_equal(g, r, f"{what} steps")
    pg, pr = g.particles(), r.particles()
    same(pg, pr, f"{what} steps")
    if tangents:
        exact(pg["D"], pr["D"], f"{what} tangents")
    del pg, pr
    g.annihilate()
    r.annihilate()
    say(f"{what}: annihilated n={r.count()}")
    stats_equal(g, r, f"{what} annihilation")
    pg, pr = g.particles(), r.particles()
    same(pg, pr, f"{what} annihilation")
    if tangents:
        exact(pg["D"], pr["D"], f"{what} tangents after annihilation")
        del pg, pr
        assert g.count(ghost=True) == r.count(ghost=True)
        gg, gr = g.particles(ghost=True), r.particles(ghost=True)
        same(gg, gr, f"{what} ghosts")
        exact(gg["D"], gr["D"], f"{what} ghost tangents")
        exact(g.density_tangent().cpu().numpy(), r.density_tangent(), f"{what} tangent density")
        gv = np.cos(np.linspace(0.0, 3.0, cfg["density"]["nbins"]))
        exact(g.density_vjp(__import__("torch").tensor(gv)).cpu().numpy(), r.density_vjp(gv), f"{what} vjp")
    else:
        del pg, pr
    assert np.array_equal(g.density().cpu().numpy(), r.density())
    say(f"{what}: done")


@pytest.mark.timeout(600)
def test_headline_sp1_1e7(P, O):
    """The benchmark's headline workload: Gaussian barrier, 1e7 particles,
    2000 x 512 grid, one 10-step epoch."""
    epoch_parity(P, O, W.gaussian_barrier_large("sp1"), 10, "sp1 1e7")


@pytest.mark.timeout(600)
def test_sp2_1e7(P, O):
    epoch_parity(P, O, W.gaussian_barrier_large("sp2"), 10, "sp2 1e7")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("strategy,mode", [("sp1", 1), ("sp1", 2), ("sp2", 1)])
def test_differentiation_1e7(P, O, strategy, mode):
    epoch_parity(P, O, W.differentiation(track_tangent=mode, strategy=strategy), 10,
                 f"differentiation {strategy} mode {mode}", tangents=True)


@pytest.mark.timeout(600)
def test_helium_4d_1e7(P, O):
    epoch_parity(P, O, W.helium_soft_coulomb(), 2, "helium 4d 1e7")


def _single(cfg, b):
    """Instance b of a batched workload as a one-instance workload drawing
    with instance b's key."""
    one = W.scaled(cfg, B=1, instance_offset=b)
    one["N0"] = cfg["N0"][b:b + 1].copy()
    one["components"] = [dict(cfg["components"][0])]
    for key in ("H", "width", "center"):
        one["components"][0][key] = cfg["components"][0][key][b:b + 1].copy()
    return one


@pytest.mark.timeout(600)
def test_batched_256_sampled_instances(P, O):
    """The batched form as bench.py runs it: a stream of its own, the
    autotuner's steps, then graph-replayed epochs.  Sampled instances (the
    largest, the smallest and two others) are replayed by the oracle alone."""
    import torch
    cfg = W.batched_barriers()
    s = torch.cuda.Stream()
    g = P.Simulation(cfg, stream=s)
    chosen = g.autotune(1)
    n = g.stats(0)["step"]
    pad = (-n) % 10
    g.step(pad)
    g.annihilate()
    g.run(20, 10, use_graph=True)
    g.synchronize()
    say(f"batched 256: autotune {chosen} after {n} steps; {n + pad + 20} steps in all")
    big, small = int(np.argmax(cfg["N0"])), int(np.argmin(cfg["N0"]))
    dg = g.density().cpu().numpy()
    for b in (big, small, 7, 200):
        r = O.OracleSim(_single(cfg, b))
        r.step(n + pad)
        r.annihilate()
        r.run(20, 10)
        stats_equal(g, r, f"batched instance {b}", b=b, rb=0)
        same(g.particles(b), r.particles(0), f"batched instance {b}")
        assert np.array_equal(dg[b], r.density()[0])
        say(f"batched 256: instance {b} (N0={int(cfg['N0'][b])}) n={r.count()} equal")
