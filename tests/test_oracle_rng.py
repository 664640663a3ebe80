"""Pins for the oracle's random-number layer.

Philox4x32-10 is checked against an implementation the oracle does not share:
rocRAND's host-side engine, driven with explicit (key, counter) tuples.  The
53-bit uniform mapping is checked on its edge values and for uniformity.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _rocrand_kat(tuples):
    hipcc = shutil.which("hipcc")
    if hipcc is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "kat")
    subprocess.check_call([hipcc, "-I/opt/rocm/include", "-O1",
                           os.path.join(HERE, "golden", "philox_rocrand_kat.cpp"), "-o", exe],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    inp = "\n".join(" ".join(str(v) for v in t) for t in tuples) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    shutil.rmtree(d, ignore_errors=True)
    return [list(map(int, l.split())) for l in out.strip().splitlines()]


def test_philox_matches_rocrand(oracle_mod):
    rng = np.random.default_rng(12345)
    tuples = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6, (5, 7, 1, 2, 3, 4)]
    tuples += [tuple(int(v) for v in rng.integers(0, 2**32, size=6)) for _ in range(200)]
    ref = _rocrand_kat(tuples)
    for t, r in zip(tuples, ref):
        got = oracle_mod.philox(t[2:], t[:2])
        assert list(map(int, got)) == r, (t, got, r)


def test_u01_edges(oracle_mod):
    u01 = oracle_mod.lib().orc_u01
    assert u01(0, 0) == 0.0
    assert u01(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert u01(0, 0x80000000) == 0.5
    # the low 11 bits of the 64-bit word are discarded
    assert u01(0x7FF, 0) == 0.0 and u01(0x800, 0) == 2.0 ** -53


def test_u01_uniform(oracle_mod):
    u01 = oracle_mod.lib().orc_u01
    vals = []
    for i in range(20000):
        w = oracle_mod.philox([i, 0, 7, 0], [0, 3])
        vals.append(u01(int(w[0]), int(w[1])))
        vals.append(u01(int(w[2]), int(w[3])))
    ks = stats.kstest(vals, "uniform")
    assert ks.pvalue > 1e-3
