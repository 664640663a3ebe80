"""Throughput of the signed-particle Wigner branching random walk on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-forms]

Headline workload: the Gaussian barrier V = 0.3 exp(-x^2/2) with 1e7 initial
signed particles (capacity 2e8), dt = 0.1, annihilation every 10 steps on a
2000 x 512 grid over x in [-200,200), k in [-8,8), density on 2000 bins, sp1
(pair generation).  A timed step is one time step of every particle (clock,
free flight, jumps and offspring families); every 10th step is followed by the
annihilation and the density readout, which are inside the timed region.
value = sum over timed steps of the particles held at the start of the step,
divided by the wall time.  Inputs are resident on the GPU before timing starts.
The timed region carries no instrumentation; the same number of steps is then
run again with HIP events around every stage (on the launch stream), and the
per-kernel durations of the roofline entry come from that second pass.

Printed: one JSON line on stdout (everything else goes to stderr).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
ANN_EVERY = 10


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stream_bytes_per_particle_step(dim):
    """Algorithmic HBM bytes of the streaming pass per particle-step: read
    x, k (f64 per axis) and the lineage id (u64), write x."""
    return dim * 8 * 2 + 8 + dim * 8


def run_form(P, torch, cfg, steps, warmup, every=ANN_EVERY, use_graph=False, density=True,
             autotune=False):
    """Runs warmup (and the autotuner), then `steps` timed steps; returns a dict
    of measurements."""
    s = torch.cuda.Stream()
    sim = P.Simulation(cfg, stream=s)
    done = 0
    tuned = None

    def advance(n):
        nonlocal done
        for _ in range(n):
            sim.step(1)
            done += 1
            if every and done % every == 0:
                sim.annihilate()
                if density:
                    sim.density()

    advance(warmup)
    if autotune:
        tuned = sim.autotune(1)
        done = sim.stats(0)["step"]
        # re-align with the annihilation schedule before timing
        while every and done % every:
            advance(1)
    s.synchronize()

    def timed(n):
        ps0 = sum(sim.stats(b)["particle_steps"] for b in range(sim.B))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if use_graph:
            sim.run(n, every, use_graph=True)
        else:
            advance(n)
        s.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, sum(sim.stats(b)["particle_steps"] for b in range(sim.B)) - ps0

    # the timed region: exactly `steps` steps with no instrumentation
    wall, ps = timed(steps)
    # the same number of steps again with HIP events around every stage on
    # the launch stream, for the per-kernel durations
    sim.profile(True)
    _, ps_prof = timed(steps)
    prof = sim.profile_read()
    sim.profile(False)
    stats = [sim.stats(b) for b in range(sim.B)]
    out = {"wall_s": wall, "particle_steps": int(ps), "rate": ps / wall,
           "prof_particle_steps": int(ps_prof),
           "n_end": int(sum(st["n"] for st in stats)), "profile": prof, "sim": sim,
           "tuned": tuned}
    return out


def roofline_of(res, dim):
    ms, launches = res["profile"]["stream"]
    if launches == 0 or ms <= 0:
        return None
    bytes_total = stream_bytes_per_particle_step(dim) * res["prof_particle_steps"]
    achieved = bytes_total / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": "k_stream",
            "avg_launch_us": round(ms * 1e3 / launches, 3),
            "bytes_per_launch": int(bytes_total / launches),
            "bytes_per_particle_step": stream_bytes_per_particle_step(dim)}


def copy_rate(torch):
    """Read+write rate of a plain 1 GiB device-to-device copy on the same GPU
    (torch's copy kernel, HIP events): what a streaming kernel can reach on
    this part in practice, beside the nominal peak."""
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    best = None
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(4):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        gbs = 4 * 2 * (1 << 30) / (e0.elapsed_time(e1) * 1e-3) / 1e9
        best = gbs if best is None else max(best, gbs)
    del a, b
    torch.cuda.empty_cache()
    return best


def measured_traffic(dim, bytes_per_launch):
    """HBM bytes per launch from the committed counter summary of k_stream,
    only if that summary was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "k_stream_traffic.json")
    if not os.path.exists(path):
        return None
    info = json.load(open(path))
    h = hashlib.sha256()
    for f in ("wbrw_stream.hpp", "wbrw_math.hpp", "wbrw_dev.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1709_02121_amd", "csrc", f), "rb").read())
    if info.get("source_sha256") != h.hexdigest():
        return None
    per = info.get("hbm_bytes_per_particle_step")
    if per is None:
        return None
    return int(per * bytes_per_launch / stream_bytes_per_particle_step(dim))


def cpu_baseline():
    """The FP64 oracle on one host core: the headline workload's physics and
    grid with 1e6 initial particles for 100 steps (annihilation every 10)."""
    import workloads as W
    from oracle import oracle as O
    O.build()
    cfg = W.scaled(W.gaussian_barrier_large("sp1"), N0=1_000_000)
    sim = O.OracleSim(cfg)
    ps = 0
    t0 = time.perf_counter()
    for s in range(100):
        ps += sim.count()
        sim.step(1)
        if (s + 1) % ANN_EVERY == 0:
            sim.annihilate()
            sim.density()
    wall = time.perf_counter() - t0
    return {"value": round(ps / wall, 1), "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": "Gaussian barrier, 2000x512 grid, 1e6 initial particles, 100 steps with "
                      "annihilation + density every 10 (%.3g particle-steps in %.1f s)" % (ps, wall)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--forms", default="all",
                    help="comma-separated forms to run besides the main line (default: all)")
    ap.add_argument("--calibrate", action="store_true",
                    help="first copy 1 GiB device to device (a reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "path is a design (histogram merge over RCCL) that this build does not run.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1709_02121_amd as P
    import workloads as W

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    P.lib()
    dev = torch.cuda.get_device_properties(0)
    log(f"device: {dev.name}, {dev.multi_processor_count} CUs")

    if args.calibrate:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        del a, b
    cfg = W.gaussian_barrier_large("sp1")
    main_res = run_form(P, torch, cfg, args.steps, args.warmup)
    roof = roofline_of(main_res, 1)
    if roof is not None:
        roof["traffic"] = measured_traffic(1, roof["bytes_per_launch"])
        cr = copy_rate(torch)
        roof["attainable"] = {"what": "plain 1 GiB device copy, read + write, same GPU",
                              "GBps": round(cr, 1), "frac": round(roof["achieved"] / cr, 4)}
    step_ms = main_res["profile"]["stream"][0] + main_res["profile"]["family"][0]
    log(f"sp1 1e7: {main_res['rate']:.4g} particle-steps/s, n_end={main_res['n_end']}, "
        f"profile={ {k: (round(v[0], 3), v[1]) for k, v in main_res['profile'].items()} }")
    main_res.pop("sim")

    forms = {"plain_sp1": {"value": round(main_res["rate"], 1),
                           "step_kernels_only": round(main_res["prof_particle_steps"] / (step_ms * 1e-3), 1)
                           if step_ms > 0 else None}}
    if not args.no_forms:
        for name, maker, steps, warm in (
                ("sp2", lambda: W.gaussian_barrier_large("sp2"), 50, 10),
                ("batched_256", lambda: W.batched_barriers(), 100, 10),
                ("fwd_adjoint", lambda: W.differentiation(), 50, 10),
                ("fwd_adjoint_x0_deriv_pairs", lambda: W.differentiation(track_tangent=2), 50, 10),
                ("fwd_adjoint_sp2", lambda: W.differentiation(strategy="sp2"), 50, 10),
                ("helium_4d", lambda: W.helium_soft_coulomb(), 10, 0)):
            if args.forms != "all" and name not in args.forms.split(","):
                continue
            try:
                torch.cuda.empty_cache()
                batched = name == "batched_256"
                r = run_form(P, torch, maker(), steps, warm, use_graph=batched, autotune=batched)
                r.pop("sim")
                forms[name] = {"value": round(r["rate"], 1), "steps": steps,
                               "particle_steps": r["particle_steps"], "n_end": r["n_end"]}
                if r["tuned"]:
                    forms[name]["autotuned_grid"] = r["tuned"]
                if name == "helium_4d":
                    rf = roofline_of(r, 2)
                    forms[name]["stream_frac_hbm"] = rf["frac"] if rf else None
                log(f"{name}: {r['rate']:.4g} particle-steps/s")
            except Exception as e:   # report, never hide, a form that failed
                forms[name] = {"error": str(e)[:300]}
                log(f"{name}: FAILED {e}")

    cpu = None if args.no_cpu else cpu_baseline()
    if cpu:
        log(f"cpu baseline: {cpu['value']:.4g} particle-steps/s on {cpu['cores']} core")

    line = {
        "metric": "particle-steps/s at 1 GPU (plain vs batched vs fwd+adjoint) and % HBM roofline",
        "value": round(main_res["rate"], 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["wall_s"] * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "gaussian_barrier_1e7_sp1", "N0": 10_000_000, "capacity": 200_000_000,
                   "grid": "2000x512", "dt": 0.1, "annihilate_every": ANN_EVERY,
                   "density_bins": 2000, "strategy": "sp1", "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": forms,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
