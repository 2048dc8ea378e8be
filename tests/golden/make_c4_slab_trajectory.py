"""Write c4_slab_trajectory.txt: the oracle's first 18 steps of the 64^3
thermal two-stream workload's physics on a 64x4x4 slab (same cell size,
4x4x4 lattice per cell per beam, drift +-0.1, thermal spread 0.01, quadratic
shape, dt 0.2, Picard tolerance 1e-8, p_max 16; 131,072 particles), FP64.

Over these steps a grid-scale mode seeded by the thermal noise grows at about
2 omega_p, far above the largest two-stream rate of the cold-beam dispersion
relation (0.354 omega_p, Sec. 5.4), until the Picard iteration needs more
passes than p_max allows.  Per step the file holds the Picard passes, whether
the step converged, and K, W, E_total divided by the box volume.  Only the
oracle runs here.

    python tests/golden/make_c4_slab_trajectory.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2606_15035_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_slab_trajectory.txt")
STEPS = 18


def main():
    wl = W.two_stream("c4", mesh=(64, 4, 4))
    vol = wl.L[0] * wl.L[1] * wl.L[2]
    S = O.OracleSim(O.make_cfg(**wl.cfg_kwargs()), wl.np)
    S.init_particles(wl.x, wl.v, wl.q, wl.m, wl.n0)
    e = S.energy()
    rows = [(0, 0, 1, e["K"] / vol, e["W"] / vol, e["E_total"] / vol)]
    for k in range(1, STEPS + 1):
        info = S.step()
        e = S.energy()
        rows.append((k, info["iters"], int(info["converged"]), e["K"] / vol, e["W"] / vol,
                     e["E_total"] / vol))
        print(f"step {k}: {info['iters']} passes, W/E {e['W'] / e['E_total']:.3e}", flush=True)
    with open(OUT, "w") as fh:
        fh.write("# oracle: 64^3 thermal two-stream physics (quadratic, dt 0.2, tol 1e-8, FP64) "
                 "on a 64x4x4 slab\n")
        fh.write("# written by tests/golden/make_c4_slab_trajectory.py\n")
        fh.write("# step passes converged K/vol W/vol E_total/vol\n")
        for r in rows:
            fh.write(f"{r[0]:d} {r[1]:d} {r[2]:d} " + " ".join(f"{v:.17e}" for v in r[3:]) + "\n")
    print(OUT)


if __name__ == "__main__":
    main()
