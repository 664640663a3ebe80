"""ctypes front end of the FP64 CPU oracle (oracle/wbrw_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and by
the CPU-baseline leg of bench.py.  The product package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wbrw_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
MAXM = 4

KIND = {"gauss": 0, "table": 1}
STRATEGY = {"sp1": 0, "sp2": 1}


def build(force=False):
    """Compile the oracle with IEEE semantics and no FMA contraction."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared", SRC, "-o", tmp, "-lm"])
    os.replace(tmp, LIB)
    return LIB


class Config(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("strategy", C.c_int32), ("M", C.c_int32), ("B", C.c_int32),
        ("instance_offset", C.c_int32), ("track_tangent", C.c_int32),
        ("seed", C.c_uint32), ("pad0", C.c_int32),
        ("hbar", C.c_double), ("mass", C.c_double), ("dt", C.c_double),
        ("gamma0", C.c_double), ("gamma_scale", C.c_double),
        ("comp_kind", C.c_int32 * MAXM), ("comp_axis", C.c_int32 * MAXM),
        ("comp_sgn", C.c_double * MAXM), ("comp_center", C.c_double * MAXM),
        ("table", C.POINTER(C.c_double) * MAXM), ("table_n", C.c_int32 * MAXM),
        ("table_qlo", C.c_double * MAXM), ("table_qhi", C.c_double * MAXM),
        ("H", C.POINTER(C.c_double)), ("width", C.POINTER(C.c_double)),
        ("center", C.POINTER(C.c_double)), ("N0", C.POINTER(C.c_int64)),
        ("init_mean_x", C.c_double * 2), ("init_sigma_x", C.c_double * 2),
        ("init_mean_k", C.c_double * 2), ("init_sigma_k", C.c_double * 2),
        ("x_lo", C.c_double), ("x_hi", C.c_double), ("k_lo", C.c_double), ("k_hi", C.c_double),
        ("nx", C.c_int32), ("nk", C.c_int32),
        ("time_dependent", C.c_int32), ("pad1", C.c_int32),
        ("mod_a", C.c_double * MAXM), ("mod_b", C.c_double * MAXM),
        ("mod_omega", C.c_double * MAXM), ("mod_phase", C.c_double * MAXM),
        ("init_kind", C.c_int32), ("pad2", C.c_int32),
        ("init_hist", C.POINTER(C.c_double)),
        ("sampler", C.c_int32 * MAXM),
    ]


class Stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "n", "n_plus", "n_minus", "n_ghost", "net", "escaped", "killed", "pairs", "events",
        "event_cap_hits", "max_depth", "S_plus", "S_minus", "N_plus", "N_minus")] + [
        ("gamma0", C.c_double), ("step", C.c_int64), ("range_errors", C.c_int64),
        ("annihilations", C.c_int64), ("triggered", C.c_int64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        vp = C.c_void_p
        L.orc_create.restype = vp
        L.orc_create.argtypes = [C.POINTER(Config)]
        L.orc_destroy.argtypes = [vp]
        L.orc_step.argtypes = [vp, C.c_int]
        L.orc_annihilate.argtypes = [vp]
        L.orc_run_adaptive.argtypes = [vp, C.c_int, C.c_int, C.c_int64]
        L.orc_density.argtypes = [vp, C.c_int, C.c_int, C.c_double, C.c_double, vp]
        L.orc_density_tangent.argtypes = [vp, C.c_int, C.c_int, C.c_double, C.c_double, vp]
        L.orc_density_vjp.argtypes = [vp, C.c_int, C.c_int, C.c_double, C.c_double, vp, vp]
        L.orc_count.restype = C.c_int64
        L.orc_count.argtypes = [vp, C.c_int, C.c_int]
        L.orc_get.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp, vp, vp, vp]
        L.orc_set.argtypes = [vp, C.c_int, C.c_int64, vp, vp, vp, vp, vp]
        L.orc_get_stats.argtypes = [vp, C.c_int, C.POINTER(Stats)]
        L.orc_get_step.restype = C.c_uint32
        L.orc_get_step.argtypes = [vp]
        L.orc_get_gamma0.restype = C.c_double
        L.orc_get_gamma0.argtypes = [vp, C.c_int]
        L.orc_get_xi.restype = C.c_double
        L.orc_get_xi.argtypes = [vp, C.c_int, C.c_int]
        L.orc_philox.argtypes = [vp, vp, vp]
        L.orc_u01.restype = C.c_double
        L.orc_u01.argtypes = [C.c_uint32, C.c_uint32]
        for f in ("orc_dlog", "orc_dsin", "orc_dcos"):
            getattr(L, f).restype = C.c_double
            getattr(L, f).argtypes = [C.c_double]
        L.orc_bootstrap_class.argtypes = [C.c_int64, vp, C.c_uint32, C.c_uint32, C.c_uint32,
                                          C.c_uint32, vp]
        L.orc_round_cell64.restype = C.c_int64
        L.orc_round_cell64.argtypes = [C.c_uint64] * 4 + [C.c_uint32] * 3 + [C.c_uint64]
        L.orc_keep_cells.argtypes = [vp, C.c_int]
        L.orc_get_cells.argtypes = [vp, C.c_int, vp, vp, vp]
        L.orc_probe_jump.argtypes = [vp, C.c_int, C.c_int, vp, C.c_uint64, C.c_uint32,
                                     vp, vp, vp]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_ptr(c), _ptr(k), _ptr(o))
    return o


def dlog(y):
    f = lib().orc_dlog
    return np.array([f(float(v)) for v in np.ravel(y)])


def dsin(a):
    f = lib().orc_dsin
    return np.array([f(float(v)) for v in np.ravel(a)])


def dcos(a):
    f = lib().orc_dcos
    return np.array([f(float(v)) for v in np.ravel(a)])


def bootstrap_class(A, seed=0, inst=0, step=0, cls=0):
    A = np.ascontiguousarray(A, dtype=np.uint64)
    out = np.zeros(len(A), dtype=np.int64)
    lib().orc_bootstrap_class(len(A), _ptr(A), seed, inst, step, cls, _ptr(out))
    return out


def round_cell(num, den, seed=0, inst=0, step=0, cell=0):
    num, den = int(num), int(den)
    m64 = (1 << 64) - 1
    return lib().orc_round_cell64(num >> 64, num & m64, den >> 64, den & m64,
                                  seed, inst, step, cell)


class OracleSim:
    """One oracle run over a workload dict (see workloads/)."""

    def __init__(self, cfg):
        self.cfg = cfg
        self._keep = []
        B = int(cfg["B"])
        comps = cfg["components"]
        M = len(comps)
        c = Config()
        c.dim = int(cfg["dim"])
        c.strategy = STRATEGY[cfg["strategy"]]
        c.M = M
        c.B = B
        c.instance_offset = int(cfg.get("instance_offset", 0))
        c.track_tangent = int(cfg.get("track_tangent", 0))
        c.seed = int(cfg["seed"])
        c.hbar, c.mass, c.dt = float(cfg["hbar"]), float(cfg["mass"]), float(cfg["dt"])
        c.gamma0, c.gamma_scale = float(cfg["gamma0"]), float(cfg["gamma_scale"])
        H = np.zeros(B * M)
        W = np.ones(B * M)
        X0 = np.zeros(B * M)
        c.time_dependent = int(any("modulation" in comp for comp in comps))
        for m, comp in enumerate(comps):
            mod = comp.get("modulation", {"a": 1.0, "b": 0.0, "omega": 0.0, "phase": 0.0})
            c.mod_a[m], c.mod_b[m] = float(mod["a"]), float(mod["b"])
            c.mod_omega[m], c.mod_phase[m] = float(mod["omega"]), float(mod["phase"])
            c.comp_kind[m] = KIND[comp["kind"]]
            c.comp_axis[m] = int(comp["axis"])
            c.sampler[m] = 1 if comp.get("sampler", "majorant") == "rejection" else 0
            if comp["kind"] == "gauss":
                H[m::M] = comp["H"]
                W[m::M] = comp["width"]
                X0[m::M] = comp["center"]
                c.comp_sgn[m] = 1.0
            else:
                t = np.ascontiguousarray(comp["table"], dtype=np.float64)
                self._keep.append(t)
                c.table[m] = t.ctypes.data_as(C.POINTER(C.c_double))
                c.table_n[m] = len(t)
                c.table_qlo[m] = float(comp["q_lo"])
                c.table_qhi[m] = float(comp["q_hi"])
                c.comp_sgn[m] = float(comp["sgn"])
                c.comp_center[m] = float(comp["center"])
        N0 = np.ascontiguousarray(cfg["N0"], dtype=np.int64)
        self._keep += [H, W, X0, N0]
        c.H = H.ctypes.data_as(C.POINTER(C.c_double))
        c.width = W.ctypes.data_as(C.POINTER(C.c_double))
        c.center = X0.ctypes.data_as(C.POINTER(C.c_double))
        c.N0 = N0.ctypes.data_as(C.POINTER(C.c_int64))
        ini = cfg["init"]
        for d in range(2):
            c.init_mean_x[d] = ini["mean_x"][d]
            c.init_sigma_x[d] = ini["sigma_x"][d]
            c.init_mean_k[d] = ini["mean_k"][d]
            c.init_sigma_k[d] = ini["sigma_k"][d]
        g = cfg["grid"]
        c.x_lo, c.x_hi, c.nx = float(g["x_lo"]), float(g["x_hi"]), int(g["nx"])
        c.k_lo, c.k_hi, c.nk = float(g["k_lo"]), float(g["k_hi"]), int(g["nk"])
        if "init_histogram" in cfg:
            hist = np.ascontiguousarray(cfg["init_histogram"], dtype=np.float64).ravel()
            self._keep.append(hist)
            c.init_kind = 1
            c.init_hist = hist.ctypes.data_as(C.POINTER(C.c_double))
        self._c = c
        self.h = lib().orc_create(C.byref(c))
        if not self.h:
            raise ValueError("oracle refused the configuration (pair probability above 1)")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    @property
    def B(self):
        return int(self.cfg["B"])

    @property
    def step_count(self):
        return lib().orc_get_step(self.h)

    def step(self, n=1):
        lib().orc_step(self.h, int(n))

    def annihilate(self):
        lib().orc_annihilate(self.h)

    def run(self, steps, annihilate_every):
        """Steps with annihilation after every `annihilate_every` steps."""
        for s in range(steps):
            self.step(1)
            if annihilate_every and (self.step_count % annihilate_every == 0):
                self.annihilate()

    def run_adaptive(self, steps, annihilate_every, limit):
        """Steps, each followed by an annihilation if the step count is a
        multiple of annihilate_every or an instance holds more than `limit`
        particles (0 turns either rule off)."""
        lib().orc_run_adaptive(self.h, int(steps), int(annihilate_every), int(limit))

    def density(self, axis=0, nbins=None, lo=None, hi=None):
        d = self.cfg["density"]
        nbins = d["nbins"] if nbins is None else nbins
        lo = d["lo"] if lo is None else lo
        hi = d["hi"] if hi is None else hi
        out = np.zeros((self.B, nbins))
        lib().orc_density(self.h, axis, nbins, lo, hi, _ptr(out))
        return out

    def density_tangent(self, axis=0, nbins=None, lo=None, hi=None):
        d = self.cfg["density"]
        nbins = d["nbins"] if nbins is None else nbins
        lo = d["lo"] if lo is None else lo
        hi = d["hi"] if hi is None else hi
        out = np.zeros((self.B, 3, nbins))
        lib().orc_density_tangent(self.h, axis, nbins, lo, hi, _ptr(out))
        return out

    def density_vjp(self, g, axis=0, nbins=None, lo=None, hi=None):
        """sum_j g[b, j] d rho[b, j] / d theta for every instance, shape (B, 3)."""
        d = self.cfg["density"]
        nbins = d["nbins"] if nbins is None else nbins
        lo = d["lo"] if lo is None else lo
        hi = d["hi"] if hi is None else hi
        gg = np.ascontiguousarray(np.broadcast_to(np.asarray(g, dtype=np.float64), (self.B, nbins)))
        out = np.zeros((self.B, 3))
        lib().orc_density_vjp(self.h, axis, nbins, lo, hi, _ptr(gg), _ptr(out))
        return out

    def count(self, b=0, ghost=False):
        return lib().orc_count(self.h, b, int(ghost))

    def particles(self, b=0, ghost=False):
        n = self.count(b, ghost)
        dim = int(self.cfg["dim"])
        x = np.zeros((dim, n)); k = np.zeros((dim, n))
        s = np.zeros(n, dtype=np.int8); w = np.zeros(n)
        i = np.zeros(n, dtype=np.uint64); D = np.zeros((n, 3))
        lib().orc_get(self.h, b, int(ghost), _ptr(x), _ptr(k), _ptr(s), _ptr(w), _ptr(i), _ptr(D))
        return {"x": x, "k": k, "sign": s, "w": w, "id": i, "D": D}

    def set_particles(self, b, x, k, sign=None, w=None, ids=None):
        x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
        k = np.ascontiguousarray(np.atleast_2d(k), dtype=np.float64)
        n = x.shape[1]
        s = None if sign is None else np.ascontiguousarray(sign, dtype=np.int8)
        ww = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        ii = None if ids is None else np.ascontiguousarray(ids, dtype=np.uint64)
        lib().orc_set(self.h, b, n, _ptr(x), _ptr(k), _ptr(s), _ptr(ww), _ptr(ii))

    def stats(self, b=0):
        st = Stats()
        lib().orc_get_stats(self.h, b, C.byref(st))
        return st.as_dict()

    def keep_cells(self, on=True):
        """Test hook: keep each later sp2 annihilation's per-cell arrays."""
        lib().orc_keep_cells(self.h, int(on))

    def cells(self, b=0):
        """(n~+, n~-, n_nu) of the last sp2 annihilation kept by keep_cells."""
        g = self.cfg["grid"]
        nc = (int(g["nx"]) * int(g["nk"])) ** int(self.cfg["dim"])
        out = [np.zeros(nc, dtype=np.int64) for _ in range(3)]
        lib().orc_get_cells(self.h, b, *(_ptr(a) for a in out))
        return tuple(out)

    def gamma0(self, b=0):
        return lib().orc_get_gamma0(self.h, b)

    def xi(self, b=0, m=0):
        return lib().orc_get_xi(self.h, b, m)

    def probe_jump(self, b, m, x, ids, e=0):
        """Vectorised over ids: (accepted, kick, sin) of one jump at position x."""
        xx = np.ascontiguousarray(np.resize(np.asarray(x, dtype=np.float64), 2))
        acc = np.zeros(len(ids), dtype=np.int32)
        kick = np.zeros(len(ids)); sn = np.zeros(len(ids))
        a = C.c_int32(); kk = C.c_double(); ss = C.c_double()
        L = lib()
        for j, i in enumerate(ids):
            L.orc_probe_jump(self.h, b, m, _ptr(xx), int(i), e, C.byref(a), C.byref(kk), C.byref(ss))
            acc[j], kick[j], sn[j] = a.value, kk.value, ss.value
        return acc, kick, sn
