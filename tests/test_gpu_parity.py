"""GPU parity: the HIP path, called through the C ABI, against the FP64 oracle
on the same seeded inputs.  Counts, signs, ids, per-cell sums, tallies and
densities must be bit-exact; positions and wave vectors too (both sides run the
same IEEE operation sequences; the stated bound of 1e-12 relative is checked
as a fallback message only)."""
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


def assert_same_ensemble(a, b, fields=("x", "k", "sign", "w", "id"), what=""):
    for f in fields:
        if f not in a or f not in b:
            continue
        x, y = np.asarray(a[f]), np.asarray(b[f])
        assert x.shape == y.shape, (what, f, x.shape, y.shape)
        if np.array_equal(x, y):
            continue
        if x.dtype.kind == "f":
            rel = np.max(np.abs(x - y) / np.maximum(np.abs(y), 1e-300))
            bad = np.flatnonzero(x != y)
            raise AssertionError(f"{what}: {f} differs at {bad[:5]} (max rel {rel:.3e})")
        bad = np.flatnonzero(x != y)
        raise AssertionError(f"{what}: {f} differs at {bad[:5]}: {x[bad[:5]]} vs {y[bad[:5]]}")


def compare(gpu, ref, what, B=1):
    keys = ["events", "pairs", "killed", "escaped", "max_depth", "event_cap_hits"]
    if gpu.cfg["strategy"] == "sp2":
        keys += ["S_plus", "S_minus", "N_plus", "N_minus"]
    for b in range(B):
        st_g, st_o = gpu.stats(b), ref.stats(b)
        assert st_g["n"] == st_o["n"], (what, b, st_g["n"], st_o["n"])
        for key in keys:
            assert st_g[key] == st_o[key], (what, b, key, st_g[key], st_o[key])
        assert_same_ensemble(gpu.particles(b), ref.particles(b), what=f"{what} b={b}")


def test_init_parity(P, O):
    cfg = W.gaussian_barrier_small(N0=np.array([20000]))
    say("init parity: 1D, N0=20000")
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    compare(g, r, "init")
    cfg4 = W.helium_soft_coulomb(N0=np.array([5003]))
    say("init parity: 2D (4D phase space), N0=5003")
    compare(P.Simulation(cfg4), O.OracleSim(cfg4), "init4d")


@pytest.mark.parametrize("n0", [1, 2047, 2048, 2049, 20000])
def test_one_step_parity(P, O, n0):
    cfg = W.gaussian_barrier_small(N0=np.array([n0]))
    say(f"one step parity: N0={n0}")
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    g.step(1)
    r.step(1)
    compare(g, r, f"step1 n0={n0}")


def test_gaussian_barrier_full_workload(P, O):
    """1e4 particles, 100 steps, annihilation every 10 (240 x 128 grid)."""
    cfg = W.gaussian_barrier_small()
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    for ep in range(10):
        g.step(10)
        r.step(10)
        if ep in (0, 9):
            compare(g, r, f"before annihilation {ep}")
        g.annihilate()
        r.annihilate()
        say(f"barrier 1e4: epoch {ep} n={r.count()}")
        if ep in (0, 4, 9):
            compare(g, r, f"after annihilation {ep}")
    dg = g.density().cpu().numpy()
    dr = r.density()
    assert np.array_equal(dg, dr)
    st = g.stats()
    assert st["step"] == 100


def test_wider_grid_and_many_tiles(P, O):
    """2000 x 512 grid, 2e5 particles (100 streaming tiles), 30 steps."""
    cfg = W.scaled(W.gaussian_barrier_large("sp1"), N0=200_000, capacity=2_000_000)
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    g.run(30, 10)
    r.run(30, 10)
    say(f"wide grid: n={r.count()}")
    compare(g, r, "wide")
    assert np.array_equal(g.density().cpu().numpy(), r.density())


def test_batched_equals_oracle(P, O):
    cfg = W.batched_barriers(B=6, N0=np.array([0, 1, 3000, 2049, 700, 9000], dtype=np.int64))
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    g.run(25, 10)
    r.run(25, 10)
    say("batched B=6 done")
    compare(g, r, "batched", B=6)
    # instance 0 has N0 = 0: its density (sum / N0) is undefined (NaN) on both sides
    dg, dr = g.density().cpu().numpy(), r.density()
    assert np.all(np.isnan(dg[0])) and np.all(np.isnan(dr[0]))
    assert np.array_equal(dg[1:], dr[1:])


def test_xcd_count_grids_and_cost_split(P, O):
    """A coarse 40 x 32 grid under instances of 1e4 particles switches on the
    per-XCD count grids of the binning pass (7 B N_h <= sum N0); after the
    first annihilation the binning split weighs the cell-ordered front of
    every instance against the offspring appended since."""
    grid = dict(W.gaussian_barrier_small()["grid"], nx=40, nk=32)
    cfg = W.batched_barriers(B=4, N0=np.array([15000, 0, 2049, 20000], dtype=np.int64), grid=grid)
    assert 7 * 4 * 40 * 32 <= int(cfg["N0"].sum())
    say("xcd count grids: B=4 (one empty), 40 x 32 grid")
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    g.run(35, 10)
    r.run(35, 10)
    compare(g, r, "xcd grids", B=4)
    # instance 1 has N0 = 0: its density (sum / N0) is undefined on both sides
    dg, dr = g.density().cpu().numpy(), r.density()
    assert np.array_equal(np.delete(dg, 1, axis=0), np.delete(dr, 1, axis=0))


def test_more_instances_than_the_lds_tallies_hold(P, O):
    """600 small instances (some empty): the per-instance event counts and
    tallies take their global-atomic paths (more than 512 instances) and the
    one-block plans scan several chunks of instances."""
    rng = np.random.default_rng(7)
    n0 = rng.integers(0, 60, size=600).astype(np.int64)
    n0[::97] = 0
    cfg = W.batched_barriers(B=600, N0=n0)
    say("600 instances")
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    g.run(12, 10)
    r.run(12, 10)
    compare(g, r, "600 instances", B=600)


def test_helium_4d_parity(P, O):
    cfg = W.helium_soft_coulomb(N0=np.array([6000]))
    cfg["grid"] = {"x_lo": -10.0, "x_hi": 10.0, "nx": 24, "k_lo": -4.0, "k_hi": 4.0, "nk": 24}
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    for ep in range(2):
        g.step(10)
        r.step(10)
        compare(g, r, f"4d before annihilation {ep}")
        g.annihilate()
        r.annihilate()
        say(f"4d: epoch {ep} n={r.count()}")
        compare(g, r, f"4d after annihilation {ep}")
    for axis in (0, 1):
        assert np.array_equal(g.density(axis=axis).cpu().numpy(), r.density(axis=axis))


def test_graph_replay_matches_plain(P, O):
    """The step + annihilation epoch captured once and replayed: every replay,
    separated by host synchronisation and eager work, matches eager launches."""
    import torch
    cfg = W.batched_barriers(B=3, N0=np.array([500, 4000, 1200], dtype=np.int64))
    s = torch.cuda.Stream()
    a, b = P.Simulation(cfg), P.Simulation(cfg, stream=s)
    for ep in range(4):
        a.run(10, 10, use_graph=False)
        b.run(10, 10, use_graph=True)
        b.synchronize()
        for i in range(3):
            assert_same_ensemble(a.particles(i), b.particles(i), what=f"graph replay {ep}")
        assert np.array_equal(a.density().cpu().numpy(), b.density().cpu().numpy())
    say("graph replay done")
    r = O.OracleSim(cfg)
    r.run(40, 10)
    compare(b, r, "graph vs oracle", B=3)


def test_capacity_overflow_is_reported(P):
    cfg = W.gaussian_barrier_small(N0=np.array([5000]), capacity=5200)
    g = P.Simulation(cfg)
    g.step(10)
    code, _ = g.stats_code()
    assert code == P.ECAPACITY


def test_sp2_bootstrap_parity(P, O):
    """Weighted pairs, then the signed residual bootstrap and the rounded
    histogram: integer classes, copies, cell values and ensembles bit-exact."""
    cfg = W.gaussian_barrier_small(N0=np.array([6000]), strategy="sp2")
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    for ep in range(3):
        g.step(10)
        r.step(10)
        compare(g, r, f"sp2 before annihilation {ep}")
        g.annihilate()
        r.annihilate()
        say(f"sp2: epoch {ep} n={r.count()} N+={r.stats()['N_plus']} N-={r.stats()['N_minus']}")
        compare(g, r, f"sp2 after annihilation {ep}")
    assert np.array_equal(g.density().cpu().numpy(), r.density())


def test_sp2_batched_and_wide(P, O):
    cfg = W.batched_barriers(B=3, N0=np.array([2500, 40000, 9000], dtype=np.int64), strategy="sp2")
    cfg["grid"] = {"x_lo": -200.0, "x_hi": 200.0, "nx": 2000, "k_lo": -8.0, "k_hi": 8.0, "nk": 512}
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    g.run(20, 10)
    r.run(20, 10)
    say("sp2 batched done")
    compare(g, r, "sp2 batched", B=3)


def test_sp2_tiny_instances(P, O):
    """sp2 on instances of 1 to 300 particles: sign classes with no draw, one
    draw and a few (the draw guide's one- and four-bucket cases, a residual
    prefix shorter than a tile), through three annihilations."""
    n0 = np.array([1, 2, 3, 5, 8, 13, 40, 300], dtype=np.int64)
    cfg = W.batched_barriers(B=len(n0), N0=n0, strategy="sp2")
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    for ep in range(3):
        g.run(4, 4)
        r.run(4, 4)
        compare(g, r, f"sp2 tiny instances, epoch {ep}", B=len(n0))
    st = [r.stats(b) for b in range(len(n0))]
    say("sp2 tiny: n " + ", ".join(str(x["n"]) for x in st))


def _exact(a, b, what):
    """Tangents and their readouts: bit-identical.  Every sum of tangents is an
    exact 32.32 fixed-point integer sum on both sides, so the GPU's order of
    addition cannot show."""
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    if np.array_equal(a, b):
        return
    bad = np.flatnonzero(a.ravel() != b.ravel())
    rel = np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))
    raise AssertionError(f"{what}: {len(bad)} elements differ, first at {bad[:5]} (max rel {rel:.3e})")


@pytest.mark.parametrize("strategy,mode", [("sp1", 1), ("sp1", 2), ("sp2", 1)])
def test_tangent_parity(P, O, strategy, mode):
    """Tangents (sp1 mode 1: likelihood-ratio scores; sp1 mode 2: x0 by
    derivative ghost pairs, which ride in the real ensemble with sign 0 until
    the next annihilation; sp2: pathwise weight tangents): the real ensemble,
    the ghosts (count, position, id) and every tangent are bit-exact, before
    and after annihilations (cell sums of tangents are exact fixed-point
    sums), and so is the tangent density."""
    cfg = W.gaussian_barrier_small(N0=np.array([5000]), gamma0=0.45, track_tangent=mode,
                                   strategy=strategy)
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    g.step(3)
    r.step(3)
    say(f"tangent mode {mode}: 3 steps n={r.count()}")
    compare(g, r, f"tangent mode {mode} before annihilation")
    _exact(g.particles()["D"], r.particles()["D"], "real tangents before annihilation")
    g.step(7)
    r.step(7)
    for ep in range(3):
        if ep:
            g.step(10)
            r.step(10)
        g.annihilate()
        r.annihilate()
        say(f"tangent mode {mode}: epoch {ep} n={r.count()} ghosts={r.count(ghost=True)}")
        compare(g, r, f"tangent real {ep}")
        pg, pr = g.particles(), r.particles()
        _exact(pg["D"], pr["D"], f"real tangents {ep}")
        assert g.count(ghost=True) == r.count(ghost=True)
        gg, gr = g.particles(ghost=True), r.particles(ghost=True)
        assert_same_ensemble(gg, gr, what=f"ghosts {ep}")
        _exact(gg["D"], gr["D"], f"ghost tangents {ep}")
    g.step(5)
    r.step(5)
    compare(g, r, "tangent mid-epoch")
    _exact(g.particles(ghost=True)["D"], r.particles(ghost=True)["D"], "ghost tangents mid-epoch")
    _exact(g.density_tangent().cpu().numpy(), r.density_tangent(), "tangent density")


def test_density_vjp_and_autograd_match_oracle(P, O):
    """Backward kernel: g . d rho / d theta from the per-particle tangents
    (fixed-point bin sums, contracted with g in bin order) equals the oracle's
    bit for bit; the torch.autograd.Function returns the same gradient."""
    import torch
    from paper_1709_02121_amd import autograd as A
    cfg = W.gaussian_barrier_small(N0=np.array([4000]), gamma0=0.45, track_tangent=1)
    cfg["init"] = dict(cfg["init"], mean_x=[-4.0, 0.0])
    x = -60 + 0.25 + 0.5 * np.arange(240)
    g = 0.5 * (1 + np.tanh(x / 2.0))
    r = O.OracleSim(cfg)
    r.run(30, 10)
    ref = r.density_vjp(g)[0]
    # and the contraction is the tangent density's, to rounding
    J = r.density_tangent()[0]
    assert np.all(np.abs(ref - J @ g) <= 1e-12 * (np.abs(J) @ np.abs(g)))
    sim = P.Simulation(cfg)
    sim.run(30, 10)
    got = sim.density_vjp(torch.tensor(g)).cpu().numpy()[0]
    _exact(got, ref, "vjp")
    theta = torch.tensor([0.3, 1.0, 0.0], dtype=torch.float64, requires_grad=True)
    rho = A.density(theta, cfg, steps=30, annihilate_every=10)
    assert np.array_equal(rho.detach().cpu().numpy(), r.density()[0])
    (rho * torch.tensor(g, device=rho.device)).sum().backward()
    _exact(theta.grad.numpy(), ref, "autograd")


@pytest.mark.parametrize("strategy,mode", [("sp1", 2), ("sp2", 1)])
def test_autograd_other_tangent_modes_and_checkpoints(P, O, strategy, mode):
    """The autograd Function in the finite-variance x0 mode (derivative ghost
    pairs) and in sp2 (pathwise tangents): the gradient equals the oracle's
    backward contraction bit for bit.  Its checkpoints are restart points: a
    handle restored from the one at step 20 reaches the same density."""
    import torch
    from paper_1709_02121_amd import autograd as A
    cfg = W.gaussian_barrier_small(N0=np.array([4000]), gamma0=0.45, track_tangent=mode,
                                   strategy=strategy)
    cfg["init"] = dict(cfg["init"], mean_x=[-4.0, 0.0])
    x = -60 + 0.25 + 0.5 * np.arange(240)
    g = 0.5 * (1 + np.tanh(x / 2.0))
    r = O.OracleSim(cfg)
    r.run(30, 10)
    ref = r.density_vjp(g)[0]
    theta = torch.tensor([0.3, 1.0, 0.0], dtype=torch.float64, requires_grad=True)
    ckpt = []
    rho = A.density(theta, cfg, steps=30, annihilate_every=10, snapshot_every=10, checkpoints=ckpt)
    assert np.array_equal(rho.detach().cpu().numpy(), r.density()[0])
    (rho * torch.tensor(g, device=rho.device)).sum().backward()
    _exact(theta.grad.numpy(), ref, f"autograd {strategy} mode {mode}")
    assert [c[0] for c in ckpt] == [10, 20, 30]
    sim = P.Simulation(A.theta_config(cfg, [0.3, 1.0, 0.0]))
    sim.restore(ckpt[1][1])
    sim.run(10, 10)
    assert np.array_equal(sim.density().cpu().numpy()[0], r.density()[0])


def test_snapshot_restore_continues_exactly(P, O):
    cfg = W.gaussian_barrier_small(N0=np.array([3000]), gamma0=0.45, track_tangent=1)
    a = P.Simulation(cfg)
    a.run(15, 10)
    snap = a.snapshot()
    a.run(15, 10)
    b = P.Simulation(cfg)
    b.restore(snap)
    b.run(15, 10)
    for ghost in (False, True):
        pa, pb = a.particles(ghost=ghost), b.particles(ghost=ghost)
        assert_same_ensemble(pa, pb, what=f"restore ghost={ghost}")
        _exact(pa["D"], pb["D"], f"restore tangents ghost={ghost}")
    r = O.OracleSim(cfg)
    r.run(30, 10)
    compare(b, r, "restore vs oracle")


def test_restore_into_used_handle(P, O):
    """A snapshot restored into a handle that has already run annihilations of
    another trajectory continues exactly as the oracle does.  Ghost placement
    and ghost tangents depend on the look-back of the next annihilation, which
    must not accept the status words the handle wrote before the restore
    (they carry the epochs the snapshot's count would reuse)."""
    cfg = W.gaussian_barrier_small(N0=np.array([3000]), gamma0=0.45, track_tangent=1)
    a = P.Simulation(cfg)
    a.run(12, 10)
    snap_a = a.snapshot()
    c = P.Simulation(dict(cfg, seed=5))   # another trajectory to the same step
    c.run(12, 10)
    snap_c = c.snapshot()
    b = P.Simulation(cfg)
    b.restore(snap_c)
    b.run(18, 10)                 # annihilations at steps 20 and 30 of that trajectory
    b.restore(snap_a)
    b.run(18, 10)                 # the same steps again, from a's state
    r = O.OracleSim(cfg)
    r.run(30, 10)
    say(f"restore into used handle: n={r.count()} ghosts={r.count(ghost=True)}")
    compare(b, r, "restored into a used handle")
    assert b.count(ghost=True) == r.count(ghost=True)
    gg, gr = b.particles(ghost=True), r.particles(ghost=True)
    assert_same_ensemble(gg, gr, what="ghosts after restore into a used handle")
    _exact(gg["D"], gr["D"], "ghost tangents after restore into a used handle")
    _exact(b.particles()["D"], r.particles()["D"], "tangents after restore into a used handle")


@pytest.mark.parametrize("strategy,graph", [("sp1", False), ("sp1", True), ("sp2", False)])
def test_threshold_triggered_annihilation_parity(P, O, strategy, graph):
    """Sec. 5's resampling when the particle number is about to exceed a
    threshold: the device decides after every step (no host round trip, also
    replayed from a captured graph), and the ensemble, the tallies and the
    number of triggered annihilations equal the oracle's."""
    cfg = W.gaussian_barrier_small(N0=np.array([3000]), strategy=strategy)
    limit = 3400 if strategy == "sp1" else 3600
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    g.run_adaptive(40, 10, limit, use_graph=graph)
    r.run_adaptive(40, 10, limit)
    st_g, st_r = g.stats(), r.stats()
    say(f"threshold {strategy} graph={graph}: annihilations {st_r['annihilations']}, "
        f"triggered {st_r['triggered']}")
    assert 3 <= st_r["triggered"] < 40 - st_r["annihilations"] + st_r["triggered"]   # fires, not always
    assert (st_g["annihilations"], st_g["triggered"]) == (st_r["annihilations"], st_r["triggered"])
    compare(g, r, f"threshold {strategy}")
    assert np.array_equal(g.density().cpu().numpy(), r.density())


def test_threshold_triggered_annihilation_4d(P, O):
    """The 4D model, whose growth the threshold keeps below the capacity."""
    cfg = W.helium_soft_coulomb(N0=np.array([3000]))
    cfg["grid"] = {"x_lo": -10.0, "x_hi": 10.0, "nx": 12, "k_lo": -4.0, "k_hi": 4.0, "nk": 12}
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    g.run_adaptive(30, 10, 9000)
    r.run_adaptive(30, 10, 9000)
    st = r.stats()
    say(f"threshold 4d: annihilations {st['annihilations']}, triggered {st['triggered']}, n={r.count()}")
    assert st["triggered"] >= 2
    assert (g.stats()["annihilations"], g.stats()["triggered"]) == (st["annihilations"], st["triggered"])
    compare(g, r, "threshold 4d")


def test_autotune_keeps_results(P, O):
    """The autotuner's steps are real steps; any grid it picks gives the same bits."""
    cfg = W.batched_barriers(B=4, N0=np.array([3000, 100, 25000, 7000], dtype=np.int64))
    g = P.Simulation(cfg)
    chosen = g.autotune(1)
    n = g.stats()["step"]
    say(f"autotune: {chosen} after {n} steps")
    r = O.OracleSim(cfg)
    r.step(n)
    compare(g, r, "autotune", B=4)
    g.run(20, 10)
    r.run(20, 10)
    compare(g, r, "after autotune", B=4)


def test_launch_shapes_keep_results(P, O):
    """Every launch configuration the autotuner can choose (streaming block
    shape and grid, family grid, binning hash size and grid) gives the oracle's
    bits, through steps and annihilations; shapes not offered are refused."""
    cfg = W.batched_barriers(B=4, N0=np.array([3000, 100, 25000, 7000], dtype=np.int64))
    r = O.OracleSim(cfg)
    r.run(25, 10)
    d = P.Simulation(cfg).launch()
    say(f"default launch: {d}")
    shapes = [(256, 8), (128, 16), (512, 4)]
    slots = [2048, 4096, 8192]
    for i, (nt, ppt) in enumerate(shapes):
        for j, sl in enumerate(slots):
            c = dict(d, stream_threads=nt, stream_ppt=ppt, bin_slots=sl,
                     stream_blocks=max(1, d["stream_blocks"] // (1 + 3 * ((i + j) % 2))),
                     family_blocks=max(1, d["family_blocks"] // (1 + 2 * (j % 2))),
                     bin_blocks=max(1, d["bin_blocks"] // (1 + i)))
            g = P.Simulation(cfg)
            g.set_launch(c)
            assert g.launch() == c
            g.run(25, 10)
            compare(g, r, f"launch {c}", B=4)
    g = P.Simulation(cfg)
    for bad in (dict(d, stream_threads=64, stream_ppt=32), dict(d, bin_slots=1000), dict(d, family_blocks=0)):
        with pytest.raises(P.WBRWError):
            g.set_launch(bad)
    c4 = W.helium_soft_coulomb(N0=np.array([1000]))
    with pytest.raises(P.WBRWError):
        P.Simulation(c4).set_launch(dict(P.Simulation(c4).launch(), stream_threads=128, stream_ppt=16))


def test_4d_family_grids_keep_results(P, O):
    """4D family kernels keep the general walks' records past the LDS pool in
    a per-block overflow area in HBM.  The default grid, a few blocks that
    reuse their areas tile after tile, and a grid wider than the areas cover
    all give the oracle's bits (full 256-parent tiles, some 50 general walks
    each, so the pool overflows in every tile)."""
    cfg = W.helium_soft_coulomb(N0=np.array([200_000]))
    r = O.OracleSim(cfg)
    r.step(3)
    say(f"4d grids: n={r.count()}")
    d = P.Simulation(cfg).launch()
    for fb in (d["family_blocks"], 7, 1100):
        g = P.Simulation(cfg)
        g.set_launch(dict(d, family_blocks=fb))
        g.step(3)
        compare(g, r, f"4d family grid {fb}")
        del g


@pytest.mark.parametrize("strategy", ["sp1", "sp2"])
def test_time_dependent_potential_parity(P, O, strategy):
    """Remark 1: kernel evaluated at the absolute jump time (switching left barrier)."""
    cfg = W.time_dependent_barriers(N0=np.array([5000]), strategy=strategy)
    # weighted pairs at every jump: 2M gamma0 = 4 growth rate, ~e^4 per epoch
    cfg["capacity_factor"] = 8.0 if strategy == "sp1" else 200.0
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    g.run(60, 10)
    r.run(60, 10)
    say(f"time-dependent {strategy}: n={r.count()}")
    compare(g, r, f"time-dependent {strategy}")
    assert np.array_equal(g.density().cpu().numpy(), r.density())


def test_signed_histogram_init_parity(P, O):
    """Alg. 3 initial sampling of signed data (cat state), then steps with the barrier."""
    cfg = W.cat_state_barrier(N0=30_000)
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    compare(g, r, "histogram init")
    g.run(20, 10)
    r.run(20, 10)
    say(f"cat state: n={r.count()}")
    compare(g, r, "histogram init + steps")


def test_alg4_rejection_sampler_parity(P, O):
    """Alg. 4 kick sampler (xi(x) table + rejection): same tables, loops and bits."""
    cfg = W.gaussian_barrier_small(N0=np.array([6000]))
    cfg["init"] = dict(cfg["init"], mean_x=[-4.0, 0.0])
    cfg["components"][0]["sampler"] = "rejection"
    g, r = P.Simulation(cfg), O.OracleSim(cfg)
    g.run(30, 10)
    r.run(30, 10)
    say(f"alg4: n={r.count()} pairs={r.stats()['pairs']}")
    compare(g, r, "alg4 sampler")
    assert np.array_equal(g.density().cpu().numpy(), r.density())
