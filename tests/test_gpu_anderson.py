"""Anderson mixing of the Picard iterates on the GPU against the oracle's.

Both sides apply the same update (Walker and Ni 2011, mixing parameter 1) to
the same passes; the GPU forms the least-squares step from FP64 normal
equations summed over the particles, the oracle by Gram-Schmidt QR of the
difference vectors, so the mixing coefficients differ in rounding only.
Fixed-iteration steps are compared at the FP64 step tolerances (1e-12 of the
velocity, displacement, field and current scales); in tolerance mode the
iteration counts agree to one and the energy identities hold at roundoff.
"""
import numpy as np
import pytest

import oracle as O
from paper_2606_15035_amd import workloads as W
from test_gpu_parity import both, compare_states, log, small_random

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_2606_15035_amd.ecpic")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    E.lib()
    return torch


@pytest.mark.parametrize("r,m,pmax", [(1, 1, 3), (2, 1, 3), (2, 2, 4), (1, 4, 5)])
def test_fixed_iterations_match_oracle(r, m, pmax):
    wl = small_random(r, seed=11)
    g, o = both(wl, tol=0.0, pmax=pmax, anderson=m)
    for step in range(3):
        ig, io = g.picard_step(), o.step()
        assert ig["iters"] == io["iters"] == pmax + 1
        compare_states(wl, g, o, f"anderson m={m} r={r} pmax={pmax} step {step}")


@pytest.mark.parametrize("r", [1, 2])
def test_tolerance_mode_energy_and_fewer_passes(r):
    wl = small_random(r, seed=9)
    g, o = both(wl, tol=1e-11, pmax=30, diagnostics=True, anderson=1)
    gp, _ = both(wl, tol=1e-11, pmax=30, diagnostics=True)
    E0 = o.energy()["E_total"]
    n_aa = n_pic = 0
    for step in range(4):
        ig, io, ip = g.picard_step(), o.step(), gp.picard_step()
        assert ig["converged"] and io["converged"]
        assert abs(ig["iters"] - io["iters"]) <= 1, (ig, io)
        n_aa += ig["iters"]
        n_pic += ip["iters"]
        if ig["iters"] == io["iters"]:
            compare_states(wl, g, o, f"anderson r={r} tol step {step}")
        eg, eo = g.energy_diagnostics(), o.energy()
        for k in ("K", "W", "E_total"):
            assert abs(eg[k] - eo[k]) <= 1e-12 * E0, (k, eg[k], eo[k])
        assert abs(eg["R_total"]) <= 1e-13 * E0
        assert eg["RA_max"] < 1e-14 and eg["gauge_max"] < 1e-12
    log(f"r={r}: passes with Anderson {n_aa}, Picard {n_pic}")
    assert n_aa <= n_pic


def test_two_stream_16x4x4_run_with_anderson():
    """The 16x4x4 two-stream workload with depth 1 and 2: 10 steps beside the
    oracle; energy at roundoff, states agree while the instability is linear."""
    wl = W.two_stream("c1")
    for m in (1, 2):
        g, o = both(wl, diagnostics=True, anderson=m)
        E0 = o.energy()["E_total"]
        for step in range(10):
            ig, io = g.picard_step(), o.step()
            assert ig["converged"] and io["converged"]
            assert abs(ig["iters"] - io["iters"]) <= 1
            eg = g.energy_diagnostics()
            assert abs(eg["R_total"]) <= 1e-13 * E0
            assert abs(eg["E_total"] - E0) <= 1e-12 * E0
        compare_states(wl, g, o, f"c1 anderson m={m} step 10")


def test_mixed_precision_with_anderson_converges():
    wl = small_random(2, seed=13)
    cfg = E.make_config(wl.n, wl.L, wl.dt, r=2, tol=1e-9, pmax=30, precision=E.MIXED,
                        diagnostics=True, anderson=1)
    g = E.Sim(cfg, wl.np)
    g.init_particles(wl.x, wl.v, wl.q, wl.m, wl.n0)
    E0 = g.energy_diagnostics()["E_total"]
    for _ in range(3):
        info = g.picard_step()
        assert info["converged"]
        e = g.energy_diagnostics()
        # rounding the accepted velocities to FP32 bounds the per-step error
        assert abs(e["R_total"]) <= 2.0 ** -23 * E0
