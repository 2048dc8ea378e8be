"""The paper's cold two-stream demonstration on the GPU, split against unsplit.

    python -m paper_2606_15035_amd.replica [--steps 1200] [--csv PREFIX]

Runs the workload of ``workloads.paper_two_stream`` twice through the HIP
library: with orbit integrals split at every crossed knot (the conservative
method) and with one 16-point Gauss rule over each whole orbit (the paper's
unsplit comparison run).  Both runs evaluate the consistency sweep every step
and record the relative energy drift (E^n - E^0) / E^0, the step's energy
defect R_total / E, the RMS chain-rule residual R_A, the Lorenz-gauge and
Gauss residuals and the Picard passes.  Prints one JSON summary line; with
--csv writes the per-step series to PREFIX_split.csv and PREFIX_unsplit.csv.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import ecpic as E
from . import workloads as W


def run(wl, split: bool, steps: int, log_every: int = 100):
    cfg = E.make_config(wl.n, wl.L, wl.dt, r=wl.r, tol=wl.tol, pmax=wl.pmax, split=split,
                        quad_points=16, diagnostics=True)
    sim = E.Sim(cfg, wl.np)
    sim.init_particles(wl.x, wl.v, wl.q, wl.m, wl.n0)
    e0 = sim.energy_diagnostics()
    E0 = e0["E_total"]
    rows = []
    t0 = time.perf_counter()
    for k in range(steps):
        info = sim.picard_step()
        e = sim.energy_diagnostics()
        rows.append((k + 1, (e["E_total"] - E0) / E0, e["R_total"] / e["E_total"], e["RA_rms"],
                     e["gauge_max"], e["gauss_max"], info["iters"], e["K"], e["W"]))
        if log_every and (k + 1) % log_every == 0:
            print(f"{'split' if split else 'unsplit'} step {k + 1}: drift {rows[-1][1]:.3e} "
                  f"RA_rms {rows[-1][3]:.3e}", flush=True)
    wall = time.perf_counter() - t0
    a = np.array(rows)
    summary = {
        "final_drift": float(a[-1, 1]),
        "max_abs_drift": float(np.abs(a[:, 1]).max()),
        "max_abs_step_defect": float(np.abs(a[:, 2]).max()),
        "max_RA_rms": float(a[:, 3].max()),
        "max_gauge": float(a[:, 4].max()),
        "max_gauss": float(a[:, 5].max()),
        "mean_passes": float(a[:, 6].mean()),
        "W_growth": float(a[:, 8].max() / max(e0["W"], 1e-300)),
        "wall_s": wall,
    }
    return summary, a


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=1200)
    ap.add_argument("--csv", default=None)
    args = ap.parse_args()
    wl = W.paper_two_stream(args.steps)
    out = {"workload": wl.description, "particles": wl.np, "steps": args.steps, "dt": wl.dt,
           "picard_tol": wl.tol, "quad_points": 16}
    for split in (True, False):
        s, a = run(wl, split, args.steps)
        name = "split" if split else "unsplit"
        out[name] = s
        if args.csv:
            np.savetxt(f"{args.csv}_{name}.csv", a, delimiter=",",
                       header="step,drift,R_total_over_E,RA_rms,gauge_max,gauss_max,passes,K,W")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
