"""Checkpoint and restart through the C ABI (ecpic_checkpoint_save /
ecpic_checkpoint_restore): a simulation restored from a checkpoint into a new
simulation object continues exactly as the saved one does.  The mixed form is
compared bitwise (its current is an exact integer sum and every other part of
its state is independent of the order of the particles); the FP64 form within
the rounding of its FP64 atomic additions (1e-13 of each quantity's scale).
Also: checkpoints of another configuration are refused, and set_state clears
the last step's balance terms while keeping the step counter.
"""
import numpy as np
import pytest

from paper_2606_15035_amd import workloads as W

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_2606_15035_amd.ecpic")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    E.lib()
    return torch


def log(*a):
    print(*a, flush=True)


def make(wl, precision, **kw):
    cfg = E.make_config(wl.n, wl.L, wl.dt, r=wl.r, tol=wl.tol, pmax=wl.pmax,
                        precision=precision, diagnostics=True, **kw)
    return E.Sim(cfg, wl.np)


def state(sim):
    s = sim.get_state()
    return s["x"], s["v"], s["vprev"], s["fields"], sim.get_current()


@pytest.mark.parametrize("name,precision", [("c3", E.MIXED), ("random", E.MIXED),
                                            ("c1", E.FP64), ("random", E.FP64)])
def test_restart_from_a_checkpoint_continues_the_run(name, precision):
    wl = (W.two_stream(name) if name != "random" else
          W.random_plasma((8, 8, 4), (1.0, 1.0, 0.5), 5000, r=2, dt=0.25, vth=0.06,
                          drift=(0.03, -0.02, 0.01), seed=31, tol=1e-11))
    a = make(wl, precision)
    a.init_particles(wl.x, wl.v, wl.q, wl.m, wl.n0)
    for _ in range(3):
        a.picard_step()
    buf = a.checkpoint()
    ea = a.energy_diagnostics()
    pa = [a.picard_step()["iters"] for _ in range(4)]
    sa = state(a)
    b = make(wl, precision)  # a new simulation, never initialised from particles
    b.restore(buf)
    eb = b.energy_diagnostics()
    assert eb["step"] == ea["step"] == 3 and eb["K"] == ea["K"] and eb["W"] == ea["W"]
    pb = [b.picard_step()["iters"] for _ in range(4)]
    sb = state(b)
    assert pa == pb
    names = ("x", "v", "vprev", "fields", "J")
    if precision == E.MIXED:
        for nm, u, w in zip(names, sa, sb):
            assert np.array_equal(u, w), nm
        log(f"[{name} mixed] 4 steps after the restart: bitwise equal ({pa} passes)")
    else:
        errs = {nm: np.abs(u - w).max() / max(np.abs(u).max(), 1e-300)
                for nm, u, w in zip(names, sa, sb)}
        log(f"[{name} fp64] 4 steps after the restart: " +
            ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))
        assert max(errs.values()) <= 1e-13


def test_checkpoint_of_another_configuration_is_refused():
    wl = W.two_stream("c1")
    a = make(wl, E.FP64)
    a.init_particles(wl.x, wl.v, wl.q, wl.m, wl.n0)
    buf = a.checkpoint()
    other = E.Sim(E.make_config(wl.n, wl.L, wl.dt, r=2, tol=wl.tol), wl.np)
    with pytest.raises(E.EcpicError) as ei:
        other.restore(buf)
    assert ei.value.status == E.EINVAL
    bad = buf.copy()
    bad[:8] = 0
    with pytest.raises(E.EcpicError) as ei:
        make(wl, E.FP64).restore(bad)
    assert ei.value.status == E.EINVAL
    fresh = E.Sim(E.make_config(wl.n, wl.L, wl.dt, r=wl.r, tol=wl.tol), wl.np)
    with pytest.raises(E.EcpicError) as ei:
        fresh.checkpoint()  # nothing to save yet
    assert ei.value.status == E.ESTATE


def test_set_state_clears_the_last_step_balance_and_keeps_the_step_counter():
    wl = W.two_stream("c1")
    a = make(wl, E.FP64)
    a.init_particles(wl.x, wl.v, wl.q, wl.m, wl.n0)
    for _ in range(2):
        a.picard_step()
    e = a.energy_diagnostics()
    assert e["step"] == 2 and e["JE_mesh"] != 0.0 and e["work_particle"] != 0.0
    s = a.get_state()
    a.set_state(s["x"], s["v"], s["vprev"], s["fields"], wl.q, wl.m)
    e = a.energy_diagnostics()
    assert e["step"] == 2
    for k in ("R_field", "R_particle", "R_total", "JE_mesh", "work_particle", "RA_rms", "RA_max",
              "pou_max"):
        assert e[k] == 0.0, k
