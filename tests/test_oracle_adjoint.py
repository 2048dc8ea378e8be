"""The oracle's adjoint of a converged step (degree 2, split orbits), pinned
against central finite differences of the oracle's own forward step, and the
multi-step gradient of the field energy with respect to the initial
perturbation amplitudes and the beam drift, against finite differences of
whole runs.

The forward map differentiated is Algorithm 1 converged (Picard run to
roundoff), with P^n rebuilt from (x^n, v^n) by eq. discrete-canonical-relation
(equal to the stored P for every accepted state).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2606_15035_amd import workloads as W


def small_case(seed=3):
    n = (8, 4, 4)
    L = (1.0, 0.6, 0.5)
    wl = W.random_plasma(n, L, 40, r=2, dt=0.2, vth=0.08, drift=(0.05, -0.03, 0.02), seed=seed)
    F = 0.05 * W.random_fields(n, 9, seed=seed + 1)
    return wl, F


class StepMap:
    """The converged one-step map (x, v, F) -> (x', v', F') of the oracle."""

    def __init__(self, wl, pmax=60):
        self.wl = wl
        self.o = O.OracleSim(O.make_cfg(wl.n, wl.L, wl.dt, r=2, tol=0.0, pmax=pmax), wl.np)
        self.o.init_particles(wl.x, wl.v, wl.q, wl.m, 1.0)

    def __call__(self, x, v, F):
        o = self.o
        o.set_state(x, v, v, None, F, self.wl.q, self.wl.m)
        o.rebuild_P()
        o.step()
        s = o.get_state()
        return s["x"], s["v"], s["fields"]


def test_one_step_adjoint_matches_finite_differences():
    wl, F = small_case()
    f = StepMap(wl)
    x, v = wl.x.copy(), wl.v.copy()
    x1, w, F1 = f(x, v, F)
    # some orbits must cross knots for the test to cover the split pieces
    H = np.asarray(wl.L) / np.asarray(wl.n)
    u0 = x / H[:, None] + 0.5
    u1 = (x + wl.dt * 0.5 * (v + w)) / H[:, None] + 0.5
    assert np.any(np.floor(u0) != np.floor(u1))
    rng = np.random.default_rng(1)
    lx1 = rng.normal(size=x.shape)
    lv1 = rng.normal(size=v.shape)
    lF1 = rng.normal(size=F.shape)
    lx0, lv0, lF0, it = f.o.adjoint_step(x, v, w, F, lx1, lv1, lF1)
    assert 2 <= it <= 60
    Lr = np.asarray(wl.L).reshape(3, 1)

    def loss(xa, va, Fa):
        xb, vb, Fb = f(xa, va, Fa)
        dx = xb - x1
        dx -= Lr * np.round(dx / Lr)
        return np.sum(lx1 * dx) + np.sum(lv1 * vb) + np.sum(lF1 * Fb)

    h = 1e-6
    for name, lam, scale in (("x", lx0, 0.01), ("v", lv0, 0.01), ("F", lF0, 1.0)):
        for _ in range(2):
            dz = scale * rng.normal(size=lam.shape)
            args_p = [x, v, F]
            args_m = [x, v, F]
            k = "xvF".index(name)
            args_p[k] = args_p[k] + h * dz
            args_m[k] = args_m[k] - h * dz
            fd = (loss(*args_p) - loss(*args_m)) / (2 * h)
            ad = np.sum(lam * dz)
            assert abs(fd - ad) <= 1e-6 * abs(fd), (name, fd, ad)


def test_field_energy_gradient_matches_finite_differences():
    wl, F = small_case(seed=7)
    o = O.OracleSim(O.make_cfg(wl.n, wl.L, wl.dt, r=2), wl.np)
    o.init_particles(wl.x, wl.v, wl.q, wl.m, 1.0)
    o.set_state(None, None, None, None, F, wl.q, wl.m)
    g = o.field_energy_grad()
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(3):
        dF = rng.normal(size=F.shape)
        Wp = o.field_energy_of((F + h * dF)[0], (F + h * dF)[2:5], (F + h * dF)[5:8])
        Wm = o.field_energy_of((F - h * dF)[0], (F - h * dF)[2:5], (F - h * dF)[5:8])
        fd = (Wp - Wm) / (2 * h)
        assert abs(fd - np.sum(g * dF)) <= 1e-8 * abs(fd)
    # psi and rho do not enter W
    assert np.all(g[1] == 0.0) and np.all(np.abs(g[8]) == 0.0)


def two_stream_small(amps, v0):
    """16x4x4 mesh, 8 particles per cell per beam, quadratic shape: the
    two-stream geometry with velocities v_x = +-v0 + sum_m a_m sin(m k1 x)."""
    n = (16, 4, 4)
    L = (W.LX, W.LX / 4, W.LX / 4)
    base = W.two_stream("c1")
    x = base.x.copy()
    sign = np.sign(base.v[0])
    pert = sum(a * np.sin((m + 1) * W.K1 * x[0]) for m, a in enumerate(amps))
    v = np.zeros_like(x)
    v[0] = sign * v0 + pert
    dvdth = [np.sin((m + 1) * W.K1 * x[0]) for m in range(len(amps))] + [sign]
    return n, L, x, v, base.q, base.m, dvdth


def run_loss(amps, v0, steps, dt, keep=False):
    n, L, x, v, q, m, dvdth = two_stream_small(amps, v0)
    o = O.OracleSim(O.make_cfg(n, L, dt, r=2, tol=0.0, pmax=30), x.shape[1])
    o.init_particles(x, v, q, m, 1.0)
    states = []
    for _ in range(steps):
        s = o.get_state()
        states.append((s["x"], s["v"], s["fields"]))
        o.step()
    return o, o.energy()["W"], states, dvdth


def test_multi_step_parameter_gradient_matches_finite_differences():
    amps, v0, steps, dt = [1e-3, 5e-4, 2e-4], 0.1, 4, 0.1
    o, Wend, states, dvdth = run_loss(amps, v0, steps, dt)
    # backward: lambda of the last level = dW/dF; no dependence on x, v
    lF = o.field_energy_grad()
    lx = lv = None
    for k in range(steps - 1, -1, -1):
        x, v, F = states[k]
        w = states[k + 1][1] if k + 1 < steps else o.get_state()["v"]
        lx, lv, lF, _ = o.adjoint_step(x, v, w, F, lx, lv, lF)
    grad = [float(np.sum(lv[0] * g)) for g in dvdth]
    h = 1e-7
    for j in range(len(amps) + 1):
        ap, am = list(amps), list(amps)
        vp = vm = v0
        if j < len(amps):
            ap[j] += h
            am[j] -= h
        else:
            vp, vm = v0 + h, v0 - h
        fd = (run_loss(ap, vp, steps, dt)[1] - run_loss(am, vm, steps, dt)[1]) / (2 * h)
        assert abs(fd - grad[j]) <= 1e-5 * abs(fd) + 1e-12 * abs(Wend), (j, fd, grad[j])
