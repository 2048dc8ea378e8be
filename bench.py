"""Benchmark: particle-pushes per second per Picard iteration on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
                    [--no-cpu-baseline] [--json-only]

A step is one call of ecpic_picard_step(): the whole hot path (orbit current
scatter, continuity + Crank-Nicolson field solve, orbit gather +
orbit-discrete-gradient push, repeated until the Picard errors fall below the
tolerance, then the end-of-step update).  Inputs are resident in HBM before the
timed region.  The metric is N_p x (Picard passes) / wall time of the timed
steps.  One JSON line is printed at the end.

Workloads (paper_2606_15035_amd.workloads): c2 = 32^3 mesh, 2,097,152
particles, quadratic shape, FP64, tol 1e-10 (default); c1 = 16x4x4, 4096
particles, linear shape, tol 1e-12.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-pushes/s per Picard iter (FP64 vs mixed) at |dE|/E; % HBM peak"
PEAK_FP64_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
PEAK_HBM_GBS = 8000.0


def gather_flops_per_push(r: int, pieces_per_orbit: float) -> float:
    """Algorithmic FP64 operations of the gather + push kernel per
    particle-push (an FMA counts 2), as written in push_piece / point_A_acc /
    gather_push_one.  Per orbit piece (r = 2, 4-point rule, 3x3x3 nodes):
    quadrature positions and z weights 123; x weights 3 x 24; per z column
    (9) y weights and column products 28 + closing (D A)^T vbar sums 24;
    per node (27) vbar . A^n and vbar . (A^{n+1} - A^n) 11, per quadrature
    point I, b_g(s_q), B_q, B'_q 8 (6 on a column's first node), grad phi
    contraction 6: 1251; knot-merge bookkeeping 6; total 1920.  Per particle:
    two point interpolants of A (2 x 228), the momentum update and velocity
    closure (36), orbit set-up, end-point wrap, crossing set-up and error
    maxima (~66), the next pass's vbar (6) = 566.  For r = 1 (2-point rule,
    2x2x2 nodes) the same terms give 410 per piece and 256 per particle."""
    if r == 2:
        return 566.0 + pieces_per_orbit * 1920.0
    return 256.0 + pieces_per_orbit * 410.0


def gather_bytes_per_push() -> float:
    """Algorithmic HBM bytes of the gather + push kernel per particle-push
    of the plain Picard iteration: read x^n, v^n, v^{n+1,p} (3 x 24 B),
    write v^{n+1,p+1} and the next pass's vbar (2 x 24 B); the mesh fields
    (80 B per node, 2.6 MB at 32^3) stay in L2 / MALL."""
    return 120.0


# Calibrated HBM traffic per launch of k_gather_push<2> on the 32^3 /
# 2,097,152-particle workload, from FETCH_SIZE and WRITE_SIZE runs scaled by
# the same counters on a streaming kernel of known size; valid only for the
# library version it was measured on (profiles/hbm_traffic_gather_scatter_32cubed_fp64.md).
MEASURED_GATHER_TRAFFIC = {"version": "ecpic-gfx950 0.15", "workload": "c2", "bytes": 264.9e6}


def time_workload(E, wl, precision, steps, warmup, anderson=0):
    """Particle-pushes/s of `steps` timed steps of workload wl after `warmup`
    steps, in the given precision and Anderson depth; returns (value, ms/step,
    mean passes, |R_total|/E of the last step, |E - E0|/E0, profile)."""
    import torch
    cfg = E.make_config(wl.n, wl.L, wl.dt, r=wl.r, kappa=wl.kappa, sigma1=wl.sigma1,
                        sigma2=wl.sigma2, tol=wl.tol, pmax=wl.pmax, precision=precision,
                        anderson=anderson)
    sim = E.Sim(cfg, wl.np)
    sim.init_particles(wl.x, wl.v, wl.q, wl.m, wl.n0)
    E0 = sim.energy_diagnostics()["E_total"]
    for _ in range(warmup):
        sim.picard_step()
    torch.cuda.synchronize()
    sim.set_profiling(2)  # events around the gather only
    iters, rel = [], 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        iters.append(sim.picard_step()["iters"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = sim.get_profile()
    sim.set_profiling(0)
    e = sim.energy_diagnostics()  # the last step's R_total and the level's energy
    rel = abs(e["R_total"]) / e["E_total"]
    drift = abs(e["E_total"] - E0) / E0
    prof["phases"] = phase_split(sim)
    out = (wl.np * sum(iters) / wall, wall / steps * 1e3, float(np.mean(iters)), rel, drift, prof)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def phase_split(sim, steps=2):
    """Per-pass times of the scatter, field solve and gather phases from
    `steps` more steps with events around every phase (after the timed
    region: each event between two kernels idles the GPU a few us)."""
    sim.set_profiling(1)
    for _ in range(steps):
        sim.picard_step()
    p = sim.get_profile()
    sim.set_profiling(0)
    return {k: p[k]["ms"] / max(p[k]["launches"], 1) for k in ("scatter", "field_solve", "gather_push")}


def run_cpu_baseline(wl, seconds_budget=30.0):
    """The oracle (serial C, one core) on the first step of the same workload."""
    import oracle as O
    o = O.OracleSim(O.make_cfg(**wl.cfg_kwargs()), wl.np)
    o.init_particles(wl.x, wl.v, wl.q, wl.m, wl.n0)
    t0 = time.perf_counter()
    info = o.step()
    t = time.perf_counter() - t0
    return {"value": wl.np * info["iters"] / t, "unit": "particle-pushes/s", "cores": 1,
            "kind": "oracle",
            "sample": f"first Picard step of the same workload ({wl.np} particles, "
                      f"{info['iters']} passes, {t:.1f} s, serial C oracle)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision lines (32^3 and 64^3 workloads)")
    ap.add_argument("--no-anderson", action="store_true",
                    help="skip the line with Anderson mixing of the Picard iterates")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU (asked for --gpus {args.gpus}); "
              "the particle decomposition over several GPUs is designed, not implemented.",
              flush=True)
        sys.exit(2)

    import torch

    from paper_2606_15035_amd import ecpic as E
    from paper_2606_15035_amd import workloads as W

    if not os.path.exists(E.LIB_PATH):
        from paper_2606_15035_amd import build as B
        B.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    wl = W.two_stream(args.workload)
    cfg = E.make_config(wl.n, wl.L, wl.dt, r=wl.r, kappa=wl.kappa, sigma1=wl.sigma1,
                        sigma2=wl.sigma2, tol=wl.tol, pmax=wl.pmax)
    sim = E.Sim(cfg, wl.np)
    sim.init_particles(wl.x, wl.v, wl.q, wl.m, wl.n0)
    E0 = sim.energy_diagnostics()["E_total"]
    for _ in range(args.warmup):
        sim.picard_step()
    torch.cuda.synchronize()

    sim.set_profiling(2)  # HIP events around the gather only
    iters = []
    dE = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = sim.picard_step()
        iters.append(info["iters"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.get_profile()
    sim.set_profiling(0)
    wall = t1 - t0
    pushes = wl.np * sum(iters)
    value = pushes / wall

    # energy error of the run (one more step read back with the full diagnostics)
    e = sim.energy_diagnostics()
    rel_step = abs(e["R_total"]) / e["E_total"]
    drift = abs(e["E_total"] - E0) / E0

    g = prof["gather_push"]
    avg_gather_s = g["ms"] / max(g["launches"], 1) * 1e-3
    pieces_per_orbit = prof["pieces"] / max(wl.np * g["launches"], 1)
    flops = gather_flops_per_push(wl.r, pieces_per_orbit) * wl.np
    achieved_tflops = flops / avg_gather_s / 1e12
    hbm_gbs = gather_bytes_per_push() * wl.np / avg_gather_s / 1e9
    version = E.lib().ecpic_version().decode()
    traffic = None
    if (MEASURED_GATHER_TRAFFIC["version"] == version
            and MEASURED_GATHER_TRAFFIC["workload"] == args.workload):
        traffic = MEASURED_GATHER_TRAFFIC["bytes"]
    roofline = {"bound": "alu", "achieved": achieved_tflops, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved_tflops / PEAK_FP64_TFLOPS, "traffic": traffic,
                "library": version,
                "kernel": "orbit gather + push (k_gather_push<2, true>)",
                "avg_launch_ms": avg_gather_s * 1e3, "pieces_per_orbit": pieces_per_orbit,
                "hbm_algorithmic_GBs": hbm_gbs, "hbm_frac": hbm_gbs / PEAK_HBM_GBS}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.description, "mesh": list(wl.n), "particles": wl.np,
                   "spline_degree": wl.r, "dt": wl.dt, "picard_tol": wl.tol,
                   "precision": "fp64", "picard_passes_mean": float(np.mean(iters)),
                   "dE_over_E_step": rel_step, "dE_over_E_run": drift},
        # two more steps with events around every phase (outside the timed
        # region, whose gather events give the roofline)
        "phases_ms_per_pass": phase_split(sim),
        "roofline": roofline,
    }
    del sim
    torch.cuda.empty_cache()
    if not args.no_anderson:
        # the same FP64 workload with Anderson mixing (depth 1): fewer passes
        # per step, each pass a little longer (two streaming kernels)
        steps = max(5, args.steps // 2)
        print("anderson depth 1 ...", flush=True)
        v_, ms_, it_, rel_, drift_, pr_ = time_workload(E, wl, E.FP64, steps, args.warmup,
                                                        anderson=1)
        out["anderson"] = {"depth": 1, "value": v_, "unit": "particle-pushes/s",
                           "ms_per_step": ms_, "steps": steps, "warmup": args.warmup,
                           "picard_passes_mean": it_, "dE_over_E_step": rel_,
                           "dE_over_E_run": drift_,
                           "step_speedup_vs_picard": out["ms_per_step"] / ms_}
    if not args.no_mixed:
        # the same workload in the mixed form, and the 64^3 / 33.5M-particle
        # workload (mixed by definition), a few steps each
        mixed = {}
        # (the 64^3 warm-up covers the steps in which its scatter settles on
        # the chunk length that fits the tile)
        for name, steps, warm in ((args.workload, max(5, args.steps // 2), 1), ("c4", 5, 3)):
            wlm = W.two_stream(name)
            print(f"mixed precision: {name} ...", flush=True)
            v_, ms_, it_, rel_, drift_, pr_ = time_workload(E, wlm, E.MIXED, steps, warm)
            g_ = pr_["gather_push"]
            mixed[name] = {"value": v_, "unit": "particle-pushes/s", "ms_per_step": ms_,
                           "steps": steps, "warmup": warm, "particles": wlm.np,
                           "mesh": list(wlm.n), "picard_passes_mean": it_,
                           "dE_over_E_step": rel_, "dE_over_E_run": drift_,
                           "phases_ms_per_pass": pr_["phases"],
                           "pieces_per_orbit": pr_["pieces"] / max(wlm.np * g_["launches"], 1),
                           "workload": wlm.description}
        out["mixed"] = mixed
        out["mixed_vs_fp64"] = mixed[args.workload]["value"] / value
    if not args.no_cpu_baseline:
        print("cpu baseline: timing the oracle on the first step ...", flush=True)
        out["cpu_baseline"] = run_cpu_baseline(W.two_stream(args.workload))
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
