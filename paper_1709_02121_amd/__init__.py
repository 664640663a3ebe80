"""MI355X signed-particle Wigner branching random walk.

A thin ctypes binding over libwbrw.so (C ABI declared in include/wbrw.h).
Every step of the method runs in the library's HIP kernels; this module only
marshals arguments, and uses PyTorch for device memory and the current HIP
stream.  There is no CPU fallback: if the library is missing or no GPU is
visible, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libwbrw.so")
SRC_DIR = os.path.join(HERE, "csrc")
HEADER = os.path.join(ROOT, "include", "wbrw.h")
MAXM = 4

OK, EINVAL, ECAPACITY, EHIP, ESTATE, EDEPTH, ERANGE = 0, -1, -2, -3, -4, -5, -6
SP1, SP2 = 0, 1
KERNEL = {"gauss": 0, "table": 1}
STRATEGY = {"sp1": SP1, "sp2": SP2}

HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-fPIC",
               "-shared", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose=False):
    """Compile libwbrw.so for gfx950 in-tree (always recompiles)."""
    src = os.path.join(SRC_DIR, "wbrw.hip")
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, src, "-o", tmp]
    out = subprocess.run(cmd, capture_output=True, text=True)
    if out.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out.stderr[-4000:])
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, LIB)
    return LIB


class Component(C.Structure):
    _fields_ = [("kind", C.c_int32), ("axis", C.c_int32), ("sign", C.c_double),
                ("center", C.c_double), ("table", C.POINTER(C.c_double)),
                ("table_n", C.c_int32), ("modulated", C.c_int32),
                ("q_lo", C.c_double), ("q_hi", C.c_double),
                ("H", C.POINTER(C.c_double)), ("width", C.POINTER(C.c_double)),
                ("center_b", C.POINTER(C.c_double)),
                ("mod_a", C.c_double), ("mod_b", C.c_double),
                ("mod_omega", C.c_double), ("mod_phase", C.c_double),
                ("sampler", C.c_int32), ("reserved2", C.c_int32)]


class Config(C.Structure):
    _fields_ = [("dim", C.c_int32), ("strategy", C.c_int32), ("n_components", C.c_int32),
                ("n_instances", C.c_int32), ("instance_offset", C.c_int32),
                ("track_tangent", C.c_int32), ("seed", C.c_uint32),
                ("max_density_bins", C.c_int32),
                ("hbar", C.c_double), ("mass", C.c_double), ("dt", C.c_double),
                ("gamma0", C.c_double), ("gamma_scale", C.c_double),
                ("comp", Component * MAXM),
                ("N0", C.POINTER(C.c_int64)), ("capacity", C.POINTER(C.c_int64)),
                ("ghost_capacity", C.c_int64),
                ("init_mean_x", C.c_double * 2), ("init_sigma_x", C.c_double * 2),
                ("init_mean_k", C.c_double * 2), ("init_sigma_k", C.c_double * 2),
                ("init_hist", C.POINTER(C.c_double)),
                ("x_lo", C.c_double), ("x_hi", C.c_double),
                ("k_lo", C.c_double), ("k_hi", C.c_double),
                ("nx", C.c_int32), ("nk", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "n", "n_ghost", "events", "pairs", "killed", "escaped", "max_depth", "event_cap_hits",
        "step", "S_plus", "S_minus", "N_plus", "N_minus", "particle_steps")] + [
        ("gamma0", C.c_double), ("annihilations", C.c_int64), ("triggered", C.c_int64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.wbrw_workspace_size.argtypes = [C.POINTER(Config), C.POINTER(C.c_size_t)]
        L.wbrw_init.argtypes = [C.POINTER(Config), vp, C.c_size_t, vp, C.POINTER(vp)]
        L.wbrw_step.argtypes = [vp, i32]
        L.wbrw_annihilate.argtypes = [vp]
        L.wbrw_run.argtypes = [vp, i32, i32, i32]
        L.wbrw_run_adaptive.argtypes = [vp, i32, i32, i64, i32]
        L.wbrw_density.argtypes = [vp, i32, i32, C.c_double, C.c_double, vp]
        L.wbrw_density_tangent.argtypes = [vp, i32, i32, C.c_double, C.c_double, vp]
        L.wbrw_density_noalloc.argtypes = [vp, i32, i32, C.c_double, C.c_double, vp]
        L.wbrw_stats.argtypes = [vp, i32, C.POINTER(Stats)]
        L.wbrw_count.argtypes = [vp, i32, i32, C.POINTER(C.c_int64)]
        L.wbrw_export.argtypes = [vp, i32, i32, i64, vp, vp, vp, vp, vp, vp]
        L.wbrw_destroy.argtypes = [vp]
        L.wbrw_profile.argtypes = [vp, i32]
        L.wbrw_autotune.argtypes = [vp, i32, vp]
        L.wbrw_get_launch.argtypes = [vp, vp]
        L.wbrw_set_launch.argtypes = [vp, vp]
        L.wbrw_density_vjp.argtypes = [vp, i32, i32, C.c_double, C.c_double, vp, vp]
        L.wbrw_snapshot_size.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.wbrw_snapshot.argtypes = [vp, vp, C.c_size_t]
        L.wbrw_restore.argtypes = [vp, vp, C.c_size_t]
        L.wbrw_profile_read.argtypes = [vp, vp, vp]
        L.wbrw_strerror.restype = C.c_char_p
        L.wbrw_strerror.argtypes = [C.c_int]
        for f in ("wbrw_workspace_size", "wbrw_init", "wbrw_step", "wbrw_annihilate", "wbrw_run",
                  "wbrw_density", "wbrw_density_tangent", "wbrw_stats", "wbrw_count",
                  "wbrw_export", "wbrw_destroy", "wbrw_profile", "wbrw_profile_read",
                  "wbrw_density_vjp", "wbrw_snapshot_size", "wbrw_snapshot", "wbrw_restore",
                  "wbrw_autotune", "wbrw_density_noalloc", "wbrw_run_adaptive", "wbrw_get_launch",
                  "wbrw_set_launch"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


class WBRWError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {lib().wbrw_strerror(code).decode()} ({code})")


def _check(code, where):
    if code != OK:
        raise WBRWError(code, where)
    return code


def make_config(cfg):
    """wbrw_config from a workload dict; returns (Config, keepalive list)."""
    keep = []
    B = int(cfg["B"])
    c = Config()
    c.dim = int(cfg["dim"])
    c.strategy = STRATEGY[cfg["strategy"]]
    c.n_components = len(cfg["components"])
    c.n_instances = B
    c.instance_offset = int(cfg.get("instance_offset", 0))
    c.track_tangent = int(cfg.get("track_tangent", 0))
    c.seed = int(cfg["seed"])
    c.max_density_bins = int(cfg.get("max_density_bins", max(cfg["density"]["nbins"], 1)))
    c.hbar, c.mass, c.dt = float(cfg["hbar"]), float(cfg["mass"]), float(cfg["dt"])
    c.gamma0, c.gamma_scale = float(cfg["gamma0"]), float(cfg["gamma_scale"])

    def dptr(a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double))

    for m, comp in enumerate(cfg["components"]):
        q = c.comp[m]
        q.kind = KERNEL[comp["kind"]]
        q.axis = int(comp["axis"])
        q.sampler = 1 if comp.get("sampler", "majorant") == "rejection" else 0
        if comp["kind"] == "gauss":
            q.H, q.width, q.center_b = dptr(comp["H"]), dptr(comp["width"]), dptr(comp["center"])
            q.sign = 1.0
            if "modulation" in comp:
                mod = comp["modulation"]
                q.modulated = 1
                q.mod_a, q.mod_b = float(mod["a"]), float(mod["b"])
                q.mod_omega, q.mod_phase = float(mod["omega"]), float(mod["phase"])
        else:
            t = np.ascontiguousarray(comp["table"], dtype=np.float64)
            q.table = dptr(t)
            q.table_n = len(t)
            q.q_lo, q.q_hi = float(comp["q_lo"]), float(comp["q_hi"])
            q.sign, q.center = float(comp["sgn"]), float(comp["center"])
    N0 = np.ascontiguousarray(cfg["N0"], dtype=np.int64)
    if "capacity" in cfg:
        cap = np.broadcast_to(np.asarray(cfg["capacity"], dtype=np.int64), (B,)).copy()
    else:
        cap = np.maximum((N0 * float(cfg.get("capacity_factor", 8.0))).astype(np.int64), 4096)
    keep += [N0, cap]
    c.N0 = N0.ctypes.data_as(C.POINTER(C.c_int64))
    c.capacity = cap.ctypes.data_as(C.POINTER(C.c_int64))
    c.ghost_capacity = int(cfg.get("ghost_capacity", 0 if not c.track_tangent else
                                   2 * cfg["grid"]["nx"] * cfg["grid"]["nk"]))
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
        c.init_hist = dptr(np.ravel(cfg["init_histogram"]))
    return c, keep


def wbrw_workspace_size(cfg):
    c, keep = make_config(cfg)
    n = C.c_size_t()
    _check(lib().wbrw_workspace_size(C.byref(c), C.byref(n)), "wbrw_workspace_size")
    return int(n.value)


class Simulation:
    """One wbrw handle: a workload's instances resident in a torch-owned workspace."""

    def __init__(self, cfg, device="cuda:0", stream=None):
        import torch

        self.cfg = cfg
        self.torch = torch
        self.device = torch.device(device)
        c, self._keep = make_config(cfg)
        self._c = c
        nbytes = C.c_size_t()
        _check(lib().wbrw_workspace_size(C.byref(c), C.byref(nbytes)), "wbrw_workspace_size")
        self.workspace_bytes = int(nbytes.value)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(lib().wbrw_init(C.byref(c), C.c_void_p(self.workspace.data_ptr()),
                               self.workspace_bytes, C.c_void_p(self.stream.cuda_stream),
                               C.byref(h)), "wbrw_init")
        self.h = h
        self.B = int(cfg["B"])
        self.dim = int(cfg["dim"])

    def close(self):
        if getattr(self, "h", None):
            lib().wbrw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        _check(lib().wbrw_step(self.h, int(n)), "wbrw_step")

    def annihilate(self):
        _check(lib().wbrw_annihilate(self.h), "wbrw_annihilate")

    def run(self, steps, annihilate_every, use_graph=False):
        _check(lib().wbrw_run(self.h, int(steps), int(annihilate_every), int(bool(use_graph))),
               "wbrw_run")

    def run_adaptive(self, steps, annihilate_every, limit, use_graph=False):
        """Steps, each followed by an annihilation if the step count is a
        multiple of annihilate_every or the instance holds more than `limit`
        particles (decided on the device)."""
        _check(lib().wbrw_run_adaptive(self.h, int(steps), int(annihilate_every), int(limit),
                                       int(bool(use_graph))), "wbrw_run_adaptive")

    def density(self, axis=0, nbins=None, lo=None, hi=None, out=None):
        d = self.cfg["density"]
        nbins = d["nbins"] if nbins is None else nbins
        lo = d["lo"] if lo is None else lo
        hi = d["hi"] if hi is None else hi
        if out is None:
            with self.torch.cuda.stream(self.stream):
                out = self.torch.empty((self.B, nbins), dtype=self.torch.float64, device=self.device)
        _check(lib().wbrw_density(self.h, axis, nbins, lo, hi, C.c_void_p(out.data_ptr())),
               "wbrw_density")
        self._order_for_caller()
        return out

    def density_noalloc(self, out, axis=0, nbins=None, lo=None, hi=None):
        """wbrw_density_noalloc into the caller's tensor `out` (B x nbins float64
        on the device): the library allocates nothing for it."""
        d = self.cfg["density"]
        nbins = d["nbins"] if nbins is None else nbins
        lo = d["lo"] if lo is None else lo
        hi = d["hi"] if hi is None else hi
        assert out.dtype == self.torch.float64 and out.numel() == self.B * nbins and out.is_contiguous()
        _check(lib().wbrw_density_noalloc(self.h, axis, nbins, lo, hi, C.c_void_p(out.data_ptr())),
               "wbrw_density_noalloc")
        self._order_for_caller()
        return out

    def density_tangent(self, axis=0, nbins=None, lo=None, hi=None, out=None):
        d = self.cfg["density"]
        nbins = d["nbins"] if nbins is None else nbins
        lo = d["lo"] if lo is None else lo
        hi = d["hi"] if hi is None else hi
        if out is None:
            with self.torch.cuda.stream(self.stream):
                out = self.torch.empty((self.B, 3, nbins), dtype=self.torch.float64, device=self.device)
        _check(lib().wbrw_density_tangent(self.h, axis, nbins, lo, hi, C.c_void_p(out.data_ptr())),
               "wbrw_density_tangent")
        self._order_for_caller()
        return out

    def _order_for_caller(self):
        """Make results visible to work the caller enqueues on torch's current stream."""
        cur = self.torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            cur.wait_stream(self.stream)

    def density_vjp(self, g, axis=0, nbins=None, lo=None, hi=None):
        """sum_j g[b, j] d rho[b, j] / d theta for every instance, shape (B, 3)."""
        t = self.torch
        d = self.cfg["density"]
        nbins = d["nbins"] if nbins is None else nbins
        lo = d["lo"] if lo is None else lo
        hi = d["hi"] if hi is None else hi
        with t.cuda.stream(self.stream):
            g = g.to(device=self.device, dtype=t.float64).reshape(self.B, nbins).contiguous()
            out = t.empty((self.B, 3), dtype=t.float64, device=self.device)
        _check(lib().wbrw_density_vjp(self.h, axis, nbins, lo, hi, C.c_void_p(g.data_ptr()),
                                      C.c_void_p(out.data_ptr())), "wbrw_density_vjp")
        self._order_for_caller()
        return out

    LAUNCH_KEYS = ("stream_blocks", "family_blocks", "stream_threads", "stream_ppt", "bin_blocks", "bin_slots")

    def autotune(self, steps_per_candidate=1):
        """Times the streaming kernel over its block shapes and grid sizes and the
        family kernel over its grid sizes on real steps, and (plain sp1) the
        binning pass over its hash sizes and grids without changing the
        ensemble; keeps the fastest (results are unchanged by the choice).
        Returns the launch configuration (see launch())."""
        out = np.zeros(6, dtype=np.int32)
        _check(lib().wbrw_autotune(self.h, int(steps_per_candidate), out.ctypes.data_as(C.c_void_p)),
               "wbrw_autotune")
        return dict(zip(self.LAUNCH_KEYS, (int(v) for v in out)))

    def launch(self):
        """The launch configuration: grid sizes of the streaming, family and
        binning kernels, the streaming block shape and the binning hash size."""
        out = np.zeros(6, dtype=np.int32)
        _check(lib().wbrw_get_launch(self.h, out.ctypes.data_as(C.c_void_p)), "wbrw_get_launch")
        return dict(zip(self.LAUNCH_KEYS, (int(v) for v in out)))

    def set_launch(self, cfg):
        """Sets the launch configuration (a dict with launch()'s keys)."""
        v = np.array([int(cfg[k]) for k in self.LAUNCH_KEYS], dtype=np.int32)
        _check(lib().wbrw_set_launch(self.h, v.ctypes.data_as(C.c_void_p)), "wbrw_set_launch")

    def snapshot(self):
        """Device copy of the current state (a torch uint8 tensor)."""
        n = C.c_size_t()
        _check(lib().wbrw_snapshot_size(self.h, C.byref(n)), "wbrw_snapshot_size")
        buf = self.torch.empty(int(n.value), dtype=self.torch.uint8, device=self.device)
        _check(lib().wbrw_snapshot(self.h, C.c_void_p(buf.data_ptr()), int(n.value)), "wbrw_snapshot")
        return buf

    def restore(self, buf):
        _check(lib().wbrw_restore(self.h, C.c_void_p(buf.data_ptr()), buf.numel()), "wbrw_restore")

    def stats(self, b=0):
        st = Stats()
        _check(lib().wbrw_stats(self.h, b, C.byref(st)), "wbrw_stats")
        return st.as_dict()

    def stats_code(self, b=0):
        st = Stats()
        return lib().wbrw_stats(self.h, b, C.byref(st)), st.as_dict()

    def count(self, b=0, ghost=False):
        n = C.c_int64()
        _check(lib().wbrw_count(self.h, b, int(ghost), C.byref(n)), "wbrw_count")
        return int(n.value)

    def particles(self, b=0, ghost=False):
        """Copies instance b's ensemble to host numpy arrays."""
        t = self.torch
        n = self.count(b, ghost)
        dev = self.device
        x = t.empty((self.dim, n), dtype=t.float64, device=dev)
        k = t.empty((self.dim, n), dtype=t.float64, device=dev)
        ids = t.empty(n, dtype=t.int64, device=dev)
        # ghosts hold a sign (always 0) in either strategy
        sp2 = self.cfg["strategy"] == "sp2" and not ghost
        s = t.empty(n, dtype=t.int8, device=dev) if not sp2 else None
        w = t.empty(n, dtype=t.float64, device=dev) if sp2 else None
        tan = bool(self.cfg.get("track_tangent", 0))
        D = t.empty((n, 3), dtype=t.float64, device=dev) if tan else None
        p = lambda a: C.c_void_p(a.data_ptr()) if (a is not None and n > 0) else None
        _check(lib().wbrw_export(self.h, b, int(ghost), n, p(x), p(k), p(s), p(w), p(ids), p(D)),
               "wbrw_export")
        out = {"x": x.cpu().numpy(), "k": k.cpu().numpy(), "id": ids.cpu().numpy().view(np.uint64)}
        if s is not None:
            out["sign"] = s.cpu().numpy()
        if w is not None:
            out["w"] = w.cpu().numpy()
        if D is not None:
            out["D"] = D.cpu().numpy()
        return out

    def synchronize(self):
        self.stream.synchronize()

    STAGES = ("stream", "family", "bin", "scan", "regen", "bootstrap", "density", "ghost",
              "events", "place", "close", "step")

    def profile(self, enable=True, steps_only=False):
        """Start (enable) or stop HIP-event timing on the handle's stream: every
        stage and whole step, or whole steps only (two events per step)."""
        mode = 0 if not enable else (2 if steps_only else 1)
        _check(lib().wbrw_profile(self.h, mode), "wbrw_profile")

    def profile_read(self):
        """{stage: (total ms, launches)} of the kernels timed since profile(True)."""
        ms = np.zeros(len(self.STAGES))
        n = np.zeros(len(self.STAGES), dtype=np.int64)
        _check(lib().wbrw_profile_read(self.h, ms.ctypes.data_as(C.c_void_p),
                                       n.ctypes.data_as(C.c_void_p)), "wbrw_profile_read")
        return {s: (float(ms[i]), int(n[i])) for i, s in enumerate(self.STAGES)}
