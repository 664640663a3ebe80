"""The density readout that allocates nothing (wbrw_density_noalloc), called
through the C ABI, against the workspace-backed wbrw_density of the same
handle: bit-identical on two calls in a row, the second with a smaller input,
and against the oracle.  Every call on a GPU shares the library's scratch
array, so the second call must not see the first one's sums."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1709_02121_amd as P
    P.lib()
    return P


def test_noalloc_density_matches_workspace_density(P):
    import torch
    from oracle import oracle as O

    O.build()
    # first call: 2e5 particles, 2000 x 512 grid, 2000 bins
    big = W.scaled(W.gaussian_barrier_large("sp1"), N0=200_000, capacity=2_000_000)
    say("noalloc: 2e5 particles, 20 steps, 2000 bins")
    g1 = P.Simulation(big)
    g1.run(20, 10)
    ref1 = g1.density().cpu().numpy()
    out1 = torch.full((1, 2000), float("nan"), dtype=torch.float64, device="cuda")
    g1.density_noalloc(out1)
    torch.cuda.synchronize()
    assert np.array_equal(out1.cpu().numpy(), ref1)
    r1 = O.OracleSim(big)
    r1.run(20, 10)
    assert np.array_equal(ref1, r1.density())

    # second call right after: a smaller ensemble, fewer bins, 3 instances
    small = W.batched_barriers(B=3, N0=np.array([4000, 0, 2500], dtype=np.int64))
    say("noalloc: 3 instances, 6500 particles, 240 bins")
    g2 = P.Simulation(small)
    g2.run(15, 10)
    ref2 = g2.density().cpu().numpy()
    out2 = torch.full((3, 240), float("nan"), dtype=torch.float64, device="cuda")
    g2.density_noalloc(out2)
    torch.cuda.synchronize()
    got2 = out2.cpu().numpy()
    assert np.array_equal(got2[0], ref2[0]) and np.array_equal(got2[2], ref2[2])
    assert np.isnan(got2[1]).all() and np.isnan(ref2[1]).all()   # N0 = 0: density undefined
    r2 = O.OracleSim(small)
    r2.run(15, 10)
    d2 = r2.density()
    assert np.array_equal(got2[0], d2[0]) and np.array_equal(got2[2], d2[2])

    # more bins than the workspace planned for; sp2 weights; the limit
    say("noalloc: 8000 bins (above max_density_bins), sp2")
    sp2 = W.gaussian_barrier_small(N0=np.array([6000]), strategy="sp2")
    g3 = P.Simulation(sp2)
    g3.run(12, 10)
    out3 = torch.empty((1, 8000), dtype=torch.float64, device="cuda")
    g3.density_noalloc(out3, nbins=8000)
    r3 = O.OracleSim(sp2)
    r3.run(12, 10)
    assert np.array_equal(out3.cpu().numpy(), r3.density(nbins=8000))
    with pytest.raises(P.WBRWError) as e:
        g3.density_noalloc(torch.empty((1, 70000), dtype=torch.float64, device="cuda"), nbins=70000)
    assert e.value.code == P.EINVAL
