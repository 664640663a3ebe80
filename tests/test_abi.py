"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/wbrw.h declares, its structs have the layout the binding
assumes, and wbrw_workspace_size validates configurations without HIP calls."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import paper_1709_02121_amd as P
import workloads as W


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.LIB):
        P.build()
    return P.lib()


def declared_functions():
    text = open(P.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(wbrw_\w+)\s*\(", text, flags=re.M)))


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(lib, n)


def test_struct_layout_matches_binding():
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "wbrw.h"
#define O(s, f) printf(#f " %zu\n", offsetof(s, f))
int main(void) {
  printf("sizeof_config %zu\nsizeof_component %zu\nsizeof_stats %zu\n",
         sizeof(wbrw_config), sizeof(wbrw_component), sizeof(wbrw_stats_t));
  O(wbrw_config, hbar); O(wbrw_config, comp); O(wbrw_config, N0); O(wbrw_config, ghost_capacity);
  O(wbrw_config, init_mean_x); O(wbrw_config, x_lo); O(wbrw_config, nx); O(wbrw_config, nk);
  O(wbrw_component, table); O(wbrw_component, q_lo); O(wbrw_component, center_b);
  O(wbrw_stats_t, gamma0); O(wbrw_stats_t, triggered);
  return 0;
}
"""
    d = tempfile.mkdtemp()
    open(os.path.join(d, "t.c"), "w").write(src)
    subprocess.check_call(["gcc", "-I", os.path.dirname(P.HEADER), os.path.join(d, "t.c"),
                           "-o", os.path.join(d, "t")])
    vals = dict(l.split() for l in subprocess.check_output([os.path.join(d, "t")], text=True).splitlines())
    vals = {k: int(v) for k, v in vals.items()}
    assert vals["sizeof_config"] == C.sizeof(P.Config)
    assert vals["sizeof_component"] == C.sizeof(P.Component)
    assert vals["sizeof_stats"] == C.sizeof(P.Stats)
    for f in ("hbar", "comp", "N0", "ghost_capacity", "init_mean_x", "x_lo", "nx", "nk"):
        assert vals[f] == getattr(P.Config, f).offset, f
    for f in ("table", "q_lo", "center_b"):
        assert vals[f] == getattr(P.Component, f).offset, f
    assert vals["gamma0"] == P.Stats.gamma0.offset
    assert vals["triggered"] == P.Stats.triggered.offset


@pytest.mark.parametrize("name", sorted(W.ALL))
def test_workspace_size_of_every_workload(lib, name):
    cfg = W.ALL[name]()
    n = P.wbrw_workspace_size(cfg)
    assert n > 0
    # particle arrays dominate: two buffer sets of at least x, k, id per capacity
    cap = int(np.sum(P.make_config(cfg)[1][1]))
    assert n >= 2 * cap * 24


def test_invalid_configs_rejected(lib):
    bad = []
    c = W.gaussian_barrier_small(); c["dt"] = 0.0; bad.append(c)
    c = W.gaussian_barrier_small(); c["grid"] = dict(c["grid"], nx=0); bad.append(c)
    c = W.gaussian_barrier_small(); c["components"][0]["width"] = np.array([0.0]); bad.append(c)
    c = W.gaussian_barrier_small(); c["capacity"] = 10; bad.append(c)           # below N0
    c = W.gaussian_barrier_small(); c["capacity"] = 1 << 31; bad.append(c)      # too large
    c = W.gaussian_barrier_small(strategy="sp2", track_tangent=2); bad.append(c)  # pairs are sp1's
    c = W.gaussian_barrier_small(track_tangent=3); bad.append(c)
    c = W.helium_soft_coulomb(track_tangent=1); bad.append(c)                   # tangents: 1D only
    c = W.helium_soft_coulomb(); c["components"][2]["sgn"] = 0.5; bad.append(c)
    for cfg in bad:
        with pytest.raises(P.WBRWError) as e:
            P.wbrw_workspace_size(cfg)
        assert e.value.code == P.EINVAL


def _pair_probability_above_one():
    """Configurations whose pair probability xi |sin| / (2 gamma0) can pass 1."""
    out = []
    c = W.gaussian_barrier_small(gamma0=0.2); out.append(("given gamma0 below xi/2", c))   # H = 0.3
    c = W.gaussian_barrier_small(gamma_scale=0.9); out.append(("gamma_scale below 1", c))
    c = W.gaussian_barrier_small(gamma0=0.45); c = W.with_theta(c, H=0.5)
    out.append(("differentiation gamma0 with a higher barrier", c))
    c = W.helium_soft_coulomb(gamma0=1.5); out.append(("table kernel, given gamma0 below xi/2", c))
    c = W.helium_soft_coulomb(gamma_scale=0.75); out.append(("table kernel, gamma_scale below 1", c))
    return out


@pytest.mark.parametrize("case", range(5))
def test_pair_probability_above_one_rejected(lib, oracle_mod, case):
    """Remark 3 needs gamma0 >= xi_m / 2 for every component, static ones
    included: both the library and the oracle refuse a configuration that
    breaks it (the sp1 acceptance would silently cap at 1)."""
    what, cfg = _pair_probability_above_one()[case]
    with pytest.raises(P.WBRWError) as e:
        P.wbrw_workspace_size(cfg)
    assert e.value.code == P.EINVAL, what
    with pytest.raises(ValueError):
        oracle_mod.OracleSim(cfg)


def test_pair_probability_at_the_bound_accepted(lib, oracle_mod):
    for cfg in (W.gaussian_barrier_small(gamma0=0.3), W.gaussian_barrier_small(gamma_scale=1.0),
                W.helium_soft_coulomb(N0=np.array([10])), W.gaussian_barrier_small(gamma0=0.45)):
        assert P.wbrw_workspace_size(cfg) > 0
        oracle_mod.OracleSim(cfg)


def test_histogram_bytes_per_cell_match_paper():
    """Sec. 5.4: 382 MB (sp1) and 763 MB (sp2) for N_h = 100^4 integer
    histograms: 4 and 8 bytes per cell.  The workspace grows by exactly that
    much per cell for the count grids (sp1: one int32 grid; sp2: one more
    int32 grid per sign class) on top of the shared per-cell scan offsets."""
    import json
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "printed_values.json")))
    g = gold["histogram_memory_MB"]
    import math
    # the paper's figures are the byte counts rounded up to whole MiB
    assert math.ceil(g["N_h"] * 4 / 2**20) == g["sp1"]
    assert math.ceil(g["N_h"] * 8 / 2**20) == g["sp2"]
    small = W.gaussian_barrier_small(N0=np.array([16]))
    big = W.gaussian_barrier_small(N0=np.array([16]))
    big["grid"] = dict(big["grid"], nx=big["grid"]["nx"] * 2)
    cells = small["grid"]["nx"] * small["grid"]["nk"]
    per_cell = {}
    for strat in ("sp1", "sp2"):
        a = dict(small, strategy=strat)
        b = dict(big, strategy=strat)
        per_cell[strat] = (P.wbrw_workspace_size(b) - P.wbrw_workspace_size(a)) / cells
    offsets = 8  # int64 exclusive scan per cell, shared by both strategies
    assert abs(per_cell["sp1"] - (4 + offsets)) < 0.1
    assert abs(per_cell["sp2"] - per_cell["sp1"] - 8) < 0.1
