"""Differentiable time integration: the field energy after K converged steps
as a function of the initial particle velocities, with a hand-written adjoint.

``FieldEnergyAfter.apply(v0, run)`` runs K steps of Algorithm 1 on the GPU
from (x0, v0) with the initial fields of the paper's initialisation (which
depend on x0 only) and returns W^K (eq. field-energy).  Its backward pass
takes dW/dF of the last level (``ecpic_field_energy_grad``) and walks the
steps backwards with ``ecpic_adjoint_step`` (the transposed Jacobian of each
converged step), recomputing the states of a segment from a checkpoint kept
every ``checkpoint_every`` steps during the forward pass.  v^{-1} only sets
the first Picard guess, so the converged trajectory depends on v0 alone.

Everything numerical runs in the HIP library; this module only moves state
between the library and torch tensors.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import ecpic as E


@dataclass
class Run:
    """A differentiable run: configuration, fixed positions and species."""
    cfg: E.Config
    x0: np.ndarray            # (3, np) initial positions (fixed)
    q: float
    m: float
    n0: float = 1.0
    steps: int = 10
    checkpoint_every: int = 10
    adjoint_tol: float = 1e-13
    adjoint_max_iters: int = 100
    # per step: ("fwd", step, Picard passes) or ("adj", step, transposed
    # iterations, seconds of the ecpic_adjoint_step call)
    log: list = field(default_factory=list)

    def sim(self) -> E.Sim:
        if getattr(self, "_sim", None) is None:
            self._sim = E.Sim(self.cfg, self.x0.shape[1])
        return self._sim


def _state(sim):
    s = sim.get_state(device=True)  # checkpoints and recomputed states stay in HBM
    return s["x"], s["v"], s["vprev"], s["fields"]


def _step(run: Run, sim: E.Sim, k: int):
    info = sim.picard_step()
    run.log.append(("fwd", k, info["iters"]))
    if not info["converged"]:
        raise RuntimeError(f"step {k}: Picard did not converge (err_v {info['err_v']:.2e}, "
                           f"err_J {info['err_J']:.2e}); the adjoint needs converged steps")


def _field_energy_after(run: Run, v0_host: np.ndarray):
    """Forward pass: W^K, the checkpoints and dW/dF of the last level."""
    sim = run.sim()
    sim.init_particles(run.x0, v0_host, run.q, run.m, run.n0)
    checkpoints = {}
    for k in range(run.steps):
        if k % run.checkpoint_every == 0:
            checkpoints[k] = _state(sim)
        _step(run, sim, k)
    W = sim.energy_diagnostics()["W"]
    return W, checkpoints, sim.field_energy_grad()


def _backward(run: Run, checkpoints, lF):
    """lambda of v^0 given lambda of the last level's fields."""
    sim = run.sim()
    torch = sim.torch
    dev = sim.state.device
    lx = lv = None
    starts = sorted(checkpoints)
    for s in reversed(starts):
        e = min(s + run.checkpoint_every, run.steps)
        x, v, vp, F = checkpoints[s]
        sim.set_state(x, v, vp, F, run.q, run.m)
        states = [(x, v, F)]
        for k in range(s, e):
            _step(run, sim, k)
            xs, vs, _, Fs = _state(sim)
            states.append((xs, vs, Fs))
        for k in range(e - 1, s - 1, -1):
            xk, vk, Fk = states[k - s]
            w = states[k - s + 1][1]
            args = (xk, vk, w, Fk)
            torch.cuda.synchronize(dev)
            t0 = time.perf_counter()  # the call returns after its stream is synchronised
            lx, lv, lF, info = sim.adjoint_step(*args, lx, lv, lF, tol=run.adjoint_tol,
                                                max_iters=run.adjoint_max_iters)
            run.log.append(("adj", k, info["iters"], time.perf_counter() - t0))
            if not info["converged"]:
                raise RuntimeError(f"adjoint of step {k} did not converge ({info['err']:.2e})")
    return lv


def _autograd_function():
    import torch

    class FieldEnergyAfter(torch.autograd.Function):
        """W^K(v0) with the hand-written adjoint as its backward."""

        @staticmethod
        def forward(ctx, v0, run: Run):
            W, ckpt, lF = _field_energy_after(run, v0.detach().cpu().numpy())
            ctx.run = run
            ctx.ckpt = ckpt
            ctx.lF = lF
            ctx.v0_device = v0.device
            return torch.tensor(W, dtype=torch.float64, device=v0.device)

        @staticmethod
        def backward(ctx, gW):
            lv0 = _backward(ctx.run, ctx.ckpt, ctx.lF * gW.to(ctx.lF.device))
            return lv0.to(ctx.v0_device), None

    return FieldEnergyAfter


_FN = None


def field_energy_after(v0, run: Run):
    """W after run.steps converged steps from (run.x0, v0); differentiable in v0."""
    global _FN
    if _FN is None:
        _FN = _autograd_function()
    return _FN.apply(v0, run)
