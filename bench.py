"""Benchmark: particle-pushes per second per Picard iteration on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
                    [--no-cpu-baseline] [--no-mixed] [--no-anderson] [--no-adjoint]

A step is one call of ecpic_picard_step(): the whole hot path (orbit current
scatter, continuity + Crank-Nicolson field solve, orbit gather +
orbit-discrete-gradient push, repeated until the Picard errors fall below the
tolerance, then the end-of-step update).  Inputs are resident in HBM before the
timed region.  The metric is N_p x (Picard passes) / wall time of the timed
steps, taken with the library's timing off.  One JSON line is printed at the
end.

Workloads (paper_2606_15035_amd.workloads): c2 = 32^3 mesh, 2,097,152
particles, quadratic shape, FP64, tol 1e-10 (default); c1 = 16x4x4, 4096
particles, linear shape, tol 1e-12.  Beside the headline: the roofline of the
orbit gather + push kernel, the same workload with Anderson mixing, the mixed
form on the 16x4x4, 32^3 and 64^3 workloads (energy and gauge errors against
FP64 runs and the oracle), the adjoint workload's gradient, and the oracle on
the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-pushes/s per Picard iter (FP64 vs mixed) at |dE|/E; % HBM peak"
PEAK_FP64_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
PEAK_HBM_GBS = 8000.0


def algorithmic_flops_per_push(r: int, pieces_per_orbit: float, nq: int | None = None) -> float:
    """Algorithmic FP64 operations (an FMA counts 2) of the orbit gather + push
    per particle-push, every term of the method counted on its own: per orbit
    piece n_q [3 s^3 + 3 (2 s^3 + 3 s^2 + 3 s) + s^3] + 3 s^3 FMA (the
    tensor-product sums of grad phi-bar and D A with A^n, A^{n+1}), per particle
    the end-point interpolant 3 s^3 FMA and ~100 flops of breakpoints and push,
    with s = r + 1 stencil nodes per axis."""
    s = r + 1
    nq = nq or (3 * r + 2) // 2
    per_piece = nq * (3 * s ** 3 + 3 * (2 * s ** 3 + 3 * s ** 2 + 3 * s) + s ** 3) + 3 * s ** 3
    return 2.0 * 3 * s ** 3 + 100.0 + pieces_per_orbit * 2.0 * per_piece


def kernel_flops_per_push(r: int, pieces_per_orbit: float) -> float:
    """FP64 operations the kernel k_gather_push actually performs per
    particle-push (an FMA counts 2): it contracts A^n, A^{n+1} with vbar at each
    node first and sums along z columns first, so it needs fewer than the
    algorithmic count.  Per orbit piece (r = 2, 4-point rule, 3x3x3 nodes):
    quadrature positions and z weights 123; x weights 3 x 24; per z column (9)
    y weights and column products 28 + closing (D A)^T vbar sums 24; per node
    (27) vbar . A^n and vbar . (A^{n+1} - A^n) 11, per quadrature point I,
    b_g(s_q), B_q, B'_q 8 (6 on a column's first node), grad phi contraction 6:
    1251; knot-merge bookkeeping 6; total 1920.  Per particle: two point
    interpolants of A (2 x 228), the momentum update and velocity closure (36),
    orbit set-up, end-point wrap, crossing set-up and error maxima (~66), the
    next pass's vbar (6) = 566.  For r = 1 (2-point rule, 2x2x2 nodes) the same
    terms give 410 per piece and 256 per particle."""
    if r == 2:
        return 566.0 + pieces_per_orbit * 1920.0
    return 256.0 + pieces_per_orbit * 410.0


def gather_bytes_per_push(mixed: bool = False) -> float:
    """Algorithmic HBM bytes of the gather + push kernel per particle-push of
    the plain Picard iteration: read x^n, v^n, v^{n+1,p}, write v^{n+1,p+1}
    and the next pass's vbar (FP64: 5 x 24 B; mixed: x^n as a cell index and
    three FP32 offsets, FP32 v^n, FP64 iterates: 4 + 12 + 12 + 3 x 24 B); the
    mesh fields (80 B per node) stay in L2 / MALL."""
    return 100.0 if mixed else 120.0


# HBM traffic per launch of k_gather_push<2> on the 32^3 / 2,097,152-particle
# FP64 workload: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by what the
# same counters read for a streaming kernel of known size (k_finalize: fetch
# 2.00 x, write 1.00 x).  A property of the kernel: valid for the library
# versions whose particle kernels are those it was measured on (0.21 added
# the device microbenchmarks, 0.22 queues a pass's scatter ahead of the
# previous pass's read-back, 0.23 launches the cell sort as a graph, 0.24
# changed an adjoint kernel only), otherwise reported as null.
MEASURED_GATHER_TRAFFIC = {"versions": ("ecpic-gfx950 0.20", "ecpic-gfx950 0.21",
                                        "ecpic-gfx950 0.22", "ecpic-gfx950 0.23",
                                        "ecpic-gfx950 0.24"),
                           "measured_on": "ecpic-gfx950 0.20", "workload": "c2",
                           "bytes": 275.4e6,
                           "source": "profiles/hbm_traffic_gather_scatter_32cubed_fp64.md"}


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count()
    return model, n


def make_sim(E, wl, precision=None, **kw):
    cfg = E.make_config(wl.n, wl.L, wl.dt, r=wl.r, kappa=wl.kappa, sigma1=wl.sigma1,
                        sigma2=wl.sigma2, tol=wl.tol, pmax=wl.pmax,
                        precision=precision if precision is not None else E.FP64, **kw)
    sim = E.Sim(cfg, wl.np)
    sim.init_particles(wl.x, wl.v, wl.q, wl.m, wl.n0)
    return sim


def timed_steps(sim, steps, profiling=0):
    """(wall seconds, passes per step) of `steps` steps, the library's timing
    at the given level (0: off)."""
    import torch
    sim.set_profiling(profiling)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = [sim.picard_step()["iters"] for _ in range(steps)]
    torch.cuda.synchronize()
    return time.perf_counter() - t0, iters


def phase_split(sim, steps=2):
    """Per-pass times of the scatter, field solve and gather phases from
    `steps` more steps with events around every phase (outside the timed
    regions: each event between two kernels idles the GPU a few us)."""
    sim.set_profiling(1)
    for _ in range(steps):
        sim.picard_step()
    p = sim.get_profile()
    sim.set_profiling(0)
    return {k: p[k]["ms"] / max(p[k]["launches"], 1) for k in ("scatter", "field_solve", "gather_push")}


def gather_roofline(E, wl, sim, steps, mixed=False):
    """Roofline of the orbit gather + push over a timed region of `steps` steps
    with HIP events around the gather on the simulation's stream."""
    sim.set_profiling(2)
    for _ in range(steps):
        sim.picard_step()
    prof = sim.get_profile()
    sim.set_profiling(0)
    g = prof["gather_push"]
    avg_s = g["ms"] / max(g["launches"], 1) * 1e-3
    ppo = prof["pieces"] / max(wl.np * g["launches"], 1)
    achieved = algorithmic_flops_per_push(wl.r, ppo) * wl.np / avg_s / 1e12
    kernel = kernel_flops_per_push(wl.r, ppo) * wl.np / avg_s / 1e12
    hbm = gather_bytes_per_push(mixed) * wl.np / avg_s / 1e9
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "flops_per_push": algorithmic_flops_per_push(wl.r, ppo),
            "kernel_flops_per_push": kernel_flops_per_push(wl.r, ppo),
            "kernel_count_achieved": kernel, "kernel_count_frac": kernel / PEAK_FP64_TFLOPS,
            "avg_launch_ms": avg_s * 1e3, "launches": g["launches"], "steps": steps,
            "pieces_per_orbit": ppo, "hbm_algorithmic_GBs": hbm, "hbm_frac": hbm / PEAK_HBM_GBS}


def run_workload(E, wl, precision, steps, warmup, anderson=0, roofline=False, fp64_ref=None):
    """Particle-pushes/s of `steps` timed steps after `warmup` steps, energy
    error per step and over the run, constraint maxima, the phase split, and
    optionally the gather roofline; fp64_ref: E_total history of an FP64 run
    of the same workload to compare with."""
    import torch
    sim = make_sim(E, wl, precision=precision, anderson=anderson)
    E0 = sim.energy_diagnostics()["E_total"]
    hist = [E0]
    for _ in range(warmup):
        sim.picard_step()
        hist.append(sim.energy_diagnostics()["E_total"])
    wall, iters = timed_steps(sim, steps)
    e = sim.energy_diagnostics()
    out = {"value": wl.np * sum(iters) / wall, "unit": "particle-pushes/s",
           "ms_per_step": wall / steps * 1e3, "steps": steps, "warmup": warmup,
           "picard_passes_mean": float(np.mean(iters)),
           "dE_over_E_step": abs(e["R_total"]) / e["E_total"],
           "dE_over_E_run": abs(e["E_total"] - E0) / E0,
           "gauge_max": e["gauge_max"], "gauss_max": e["gauss_max"]}
    hist.append(e["E_total"])
    if fp64_ref is not None:
        out["dE_vs_fp64_after_warmup"] = abs(hist[warmup] - fp64_ref[warmup]) / fp64_ref[warmup]
    if roofline:
        out["roofline"] = gather_roofline(E, wl, sim, steps, mixed=precision == E.MIXED)
    out["phases_ms_per_pass"] = phase_split(sim)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out, hist


def mixed_c3_against_oracle(E, W):
    """The 16x4x4 workload in the mixed form, its 100 steps on the GPU beside the
    FP64 oracle's 100 steps from the same (storage-exact) state: energy error per
    step and over the run of each, the largest energy difference between them,
    and the Gauss and gauge residual maxima."""
    import oracle as O
    wl = W.two_stream("c3")
    x = wl.x.copy()
    # positions and velocities the mixed storage holds exactly
    H = (np.asarray(wl.L) / np.asarray(wl.n)).reshape(3, 1)
    c = np.floor(x / H)
    x = (c + (x / H - c).astype(np.float32).astype(np.float64)) * H
    v = wl.v.astype(np.float32).astype(np.float64)
    g = E.Sim(E.make_config(wl.n, wl.L, wl.dt, r=wl.r, tol=wl.tol, pmax=wl.pmax,
                            precision=E.MIXED, diagnostics=True), wl.np)
    g.init_particles(x, v, wl.q, wl.m, wl.n0)
    o = O.OracleSim(O.make_cfg(**wl.cfg_kwargs()), wl.np)
    o.init_particles(x, v, wl.q, wl.m, wl.n0)
    E0g, E0o = g.energy_diagnostics()["E_total"], o.energy()["E_total"]
    step_g = step_o = diff = gauge = gauss = 0.0
    for _ in range(wl.steps):
        g.picard_step()
        o.step()
        eg, eo = g.energy_diagnostics(), o.energy()
        step_g = max(step_g, abs(eg["R_total"]) / eg["E_total"])
        step_o = max(step_o, abs(eo["R_total"]) / eo["E_total"])
        diff = max(diff, abs(eg["E_total"] - eo["E_total"]) / eo["E_total"])
        gauge, gauss = max(gauge, eg["gauge_max"]), max(gauss, eg["gauss_max"])
    g.close()
    return {"workload": wl.description, "steps": wl.steps,
            "dE_over_E_step_max": step_g, "dE_over_E_run": abs(eg["E_total"] - E0g) / E0g,
            "oracle_fp64_dE_over_E_step_max": step_o,
            "oracle_fp64_dE_over_E_run": abs(eo["E_total"] - E0o) / E0o,
            "max_E_difference_vs_oracle": diff, "gauge_max": gauge, "gauss_max": gauss}


def adjoint_gradient(E, W):
    """The adjoint workload (32^3, 2,097,152 particles, quadratic shape, FP64):
    the gradient of the field energy after 50 steps (Picard tolerance 1e-13,
    checkpoints every 10) with respect to 8 mode amplitudes and the drift,
    through the torch.autograd function of the hand-written adjoint."""
    import torch

    from paper_2606_15035_amd import adjoint as AD
    base = W.two_stream("c5")
    x = base.x
    sign = np.sign(base.v[0])
    basis = np.stack([np.sin((m + 1) * W.K1 * x[0]) for m in range(8)])
    cfg = E.make_config(base.n, base.L, base.dt, r=2, tol=1e-13, pmax=40)
    run = AD.Run(cfg=cfg, x0=x, q=base.q, m=base.m, steps=base.steps, checkpoint_every=10)
    theta = torch.tensor([1e-3] * 8 + [W.V0], dtype=torch.float64, device="cuda",
                         requires_grad=True)
    b = torch.as_tensor(basis, dtype=torch.float64, device="cuda")
    sg = torch.as_tensor(sign, dtype=torch.float64, device="cuda")
    vx = sg * theta[8] + (theta[:8, None] * b).sum(0)
    z = torch.zeros_like(vx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Wk = AD.field_energy_after(torch.stack([vx, z, z]), run)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Wk.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    adj = [e for e in run.log if e[0] == "adj"]
    fwd = [e for e in run.log if e[0] == "fwd"]
    run.sim().close()
    return {"workload": base.description, "steps": base.steps, "checkpoint_every": 10,
            "gradient_s": t2 - t0, "forward_s": t1 - t0, "backward_s": t2 - t1,
            "adjoint_step_ms_mean": 1e3 * float(np.mean([e[3] for e in adj])),
            "transposed_iterations": int(sum(e[2] for e in adj)),
            "transposed_iterations_per_step": float(np.mean([e[2] for e in adj])),
            "ms_per_transposed_iteration": 1e3 * sum(e[3] for e in adj) / max(sum(e[2] for e in adj), 1),
            "forward_passes": int(sum(e[2] for e in fwd)),
            "W": float(Wk.detach()), "grad": [float(v) for v in theta.grad.cpu().numpy()]}


def run_cpu_baseline(wl):
    """The oracle (serial C, one core) on the first step of the same workload."""
    import oracle as O
    o = O.OracleSim(O.make_cfg(**wl.cfg_kwargs()), wl.np)
    o.init_particles(wl.x, wl.v, wl.q, wl.m, wl.n0)
    t0 = time.perf_counter()
    info = o.step()
    t = time.perf_counter() - t0
    model, n = host_cpu()
    return {"value": wl.np * info["iters"] / t, "unit": "particle-pushes/s", "cores": 1,
            "kind": "oracle", "host_cpu": model, "host_nproc": n,
            "sample": f"first Picard step of the same workload ({wl.np} particles, "
                      f"{info['iters']} passes, {t:.1f} s, serial C oracle on one of {n} "
                      f"host cores)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision lines (16x4x4, 32^3 and 64^3 workloads)")
    ap.add_argument("--no-anderson", action="store_true",
                    help="skip the line with Anderson mixing of the Picard iterates")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint workload's gradient")
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
    head, hist64 = run_workload(E, wl, E.FP64, args.steps, args.warmup, roofline=True)
    version = E.lib().ecpic_version().decode()
    roofline = head.pop("roofline")
    roofline["kernel"] = "orbit gather + push (k_gather_push<2, true>)"
    roofline["library"] = version
    mt = MEASURED_GATHER_TRAFFIC
    roofline["traffic"] = (mt["bytes"] if version in mt["versions"] and mt["workload"] == args.workload
                           else None)
    roofline["traffic_source"] = f"{mt['source']} ({mt['measured_on']}; not measured in this run)"
    # the device's own FP64 FMA and streaming rates, beside the published peaks
    peaks = E.measure_peaks()
    peaks["source"] = "ecpic_measure_peaks: FMA-chain kernel and streaming copy, best of 5"

    def against_measured(r):
        r["measured_peak"] = peaks
        r["frac_of_measured_fp64"] = r["achieved"] / peaks["fp64_tflops"]
        r["hbm_frac_of_measured"] = r["hbm_algorithmic_GBs"] / peaks["hbm_GBs"]
    against_measured(roofline)

    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "particle-pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.description, "mesh": list(wl.n), "particles": wl.np,
                   "spline_degree": wl.r, "dt": wl.dt, "picard_tol": wl.tol,
                   "precision": "fp64", "picard_passes_mean": head["picard_passes_mean"],
                   "dE_over_E_step": head["dE_over_E_step"], "dE_over_E_run": head["dE_over_E_run"],
                   "gauge_max": head["gauge_max"], "gauss_max": head["gauss_max"]},
        "phases_ms_per_pass": head["phases_ms_per_pass"],
        "roofline": roofline,
    }
    if not args.no_anderson:
        # the same FP64 workload with Anderson mixing (depth 1): fewer passes
        # per step, each pass a little longer (two streaming kernels)
        print("anderson depth 1 ...", flush=True)
        a, _ = run_workload(E, wl, E.FP64, max(5, args.steps // 2), args.warmup, anderson=1)
        a["depth"] = 1
        a["step_speedup_vs_picard"] = out["ms_per_step"] / a["ms_per_step"]
        out["anderson"] = a
    if not args.no_mixed:
        mixed = {}
        print(f"mixed precision: {args.workload} ...", flush=True)
        m2, _ = run_workload(E, wl, E.MIXED, max(5, args.steps // 2), args.warmup,
                             fp64_ref=hist64)
        m2["workload"] = wl.description
        mixed[args.workload] = m2
        # the 64^3 / 33.5M-particle workload (mixed by definition); the warm-up
        # covers the steps in which its scatter settles on its chunk length
        print("mixed precision: c4 ...", flush=True)
        wl4 = W.two_stream("c4")
        m4, _ = run_workload(E, wl4, E.MIXED, 5, 3, roofline=True)
        m4["roofline"]["kernel"] = "orbit gather + push (k_gather_push<2, true>, mixed store)"
        against_measured(m4["roofline"])
        m4["workload"] = wl4.description
        m4["particles"] = wl4.np
        mixed["c4"] = m4
        del wl4
        print("mixed precision: c3 beside the oracle ...", flush=True)
        mixed["c3"] = mixed_c3_against_oracle(E, W)
        out["mixed"] = mixed
        out["mixed_vs_fp64"] = m2["value"] / out["value"]
    if not args.no_adjoint:
        print("adjoint workload: gradient of W^50 ...", flush=True)
        out["adjoint"] = adjoint_gradient(E, W)
    if not args.no_cpu_baseline:
        print("cpu baseline: timing the oracle on the first step ...", flush=True)
        out["cpu_baseline"] = run_cpu_baseline(W.two_stream(args.workload))
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
