"""Seeded synthetic inputs shared by the GPU path, the tests and the oracle.

This module holds no arithmetic of the method itself: it only lays out
particles and velocities (numpy, PCG64 with a fixed seed) for the cold
two-stream problems and for random parity cases, and names the constants of
each workload.  The same arrays are handed to the HIP library and to the CPU
oracle.

Two-stream workloads follow the setup of Sec. 5.4 of the paper: mobile
electrons in two counter-streaming beams over a uniform neutralising ion
background n0 = 1, kappa = sigma1 = sigma2 = 1, q_p = -n0 |Omega| / N_p,
m_p = |q_p| (so q/m = -1 and omega_p = 1), quiet-start positions with both
beams at identical positions.  The sizes are this project's workloads (the
paper's own run is 16^3 at v0 = 0.3): the drift v0 = 0.1 and k1 v0 / omega_p = 0.6
give k1 = 6 and L_x = 2 pi / 6.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED = 2606
V0 = 0.1
K1 = 0.6 / V0
LX = 2.0 * math.pi / K1


@dataclasses.dataclass
class Workload:
    name: str
    n: tuple
    L: tuple
    dt: float
    steps: int
    r: int
    tol: float
    pmax: int
    precision: str  # "fp64" or "mixed"
    x: np.ndarray   # (3, np)
    v: np.ndarray   # (3, np)
    q: float
    m: float
    n0: float = 1.0
    kappa: float = 1.0
    sigma1: float = 1.0
    sigma2: float = 1.0
    description: str = ""
    # several species: particle i has charge qs[species[i]] and mass ms[species[i]]
    species: np.ndarray | None = None
    qs: tuple | None = None
    ms: tuple | None = None

    @property
    def np(self) -> int:
        return int(self.x.shape[1])

    def cfg_kwargs(self) -> dict:
        return dict(n=self.n, L=self.L, dt=self.dt, r=self.r, kappa=self.kappa,
                    sigma1=self.sigma1, sigma2=self.sigma2, tol=self.tol, pmax=self.pmax)


def _species(n0, L, np_):
    vol = L[0] * L[1] * L[2]
    q = -n0 * vol / np_
    return q, abs(q)


def _quiet_x_lattice(n, L, per_cell_x):
    """Cell-major quiet start: per cell, per_cell_x points along x at
    (i + (p + 1/2) / per_cell_x) H_x and the cell centre in y and z.
    Returns (3, ncell * per_cell_x), ordered cell by cell."""
    H = [L[a] / n[a] for a in range(3)]
    ix, iy, iz, p = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]),
                                np.arange(per_cell_x), indexing="ij")
    x = (ix + (p + 0.5) / per_cell_x) * H[0]
    y = (iy + 0.5) * H[1] + 0.0 * p
    z = (iz + 0.5) * H[2] + 0.0 * p
    return np.stack([x.ravel(), y.ravel(), z.ravel()])


def _quiet_3d_lattice(n, L, sub):
    """Cell-major quiet start with a sub x sub x sub lattice in every cell."""
    H = [L[a] / n[a] for a in range(3)]
    ix, iy, iz, a, b, c = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]),
                                      np.arange(sub), np.arange(sub), np.arange(sub),
                                      indexing="ij")
    x = (ix + (a + 0.5) / sub) * H[0]
    y = (iy + (b + 0.5) / sub) * H[1]
    z = (iz + (c + 0.5) / sub) * H[2]
    return np.stack([x.ravel(), y.ravel(), z.ravel()])


def two_stream(name: str, mesh: tuple | None = None) -> Workload:
    """The named two-stream workload.

    mesh: if given, the workload's physics on another mesh with the same
    cell size (the box is mesh x H): the same particles per cell at the same
    places within each cell, the same drift, perturbation, shape, dt and
    tolerance.  For c1, c2, c3 and c5 the x extent must stay (the
    perturbation is periodic in L_x); since every cell holds the same
    pattern and the perturbation depends on x alone, a slab with fewer
    y, z cells evolves exactly as the full box does, up to rounding.  c4's
    thermal velocities are drawn per particle for the mesh given.

    c1  16x4x4 mesh, 8 particles per cell per beam (4096), linear shape, FP64,
        1e-3 sin(k1 x) velocity perturbation, dt = 0.1, 100 steps, tol 1e-12
    c2  32^3 mesh, 32 per cell per beam (2,097,152), quadratic shape, FP64,
        random 1e-3 perturbation over the lowest 4 x-modes, dt = 0.1, 200 steps,
        tol 1e-10
    c3  c1 in mixed precision
    c4  64^3 mesh, 4x4x4 lattice per cell per beam (33,554,432), quadratic, mixed,
        drift plus Maxwellian spread 0.01 in every component, dt = 0.2, 100 steps,
        tol 1e-8
    c5  c2 geometry with 1e-3 amplitudes on the lowest 8 x-modes, 50 steps, FP64
    """
    rng = np.random.Generator(np.random.PCG64(SEED))
    if name in ("c1", "c3"):
        n = (16, 4, 4)
        L = (LX, LX / 4, LX / 4)
        ppb = 8
        pos = _quiet_x_lattice(n, L, ppb)
        pert = 1e-3 * np.sin(K1 * pos[0])
        dt, steps, r, tol = 0.1, 100, 1, 1e-12
        prec = "fp64" if name == "c1" else "mixed"
        desc = "cold two-stream 16x4x4, 8 ppc/beam, CIC, 1e-3 sin(k1 x)"
    elif name in ("c2", "c5"):
        n = (32, 32, 32)
        L = (LX, LX, LX)
        ppb = 32
        pos = _quiet_x_lattice(n, L, ppb)
        if name == "c2":
            eps = 1e-3 * rng.uniform(0.5, 1.0, size=4)
            th = rng.uniform(0.0, 2 * math.pi, size=4)
            pert = sum(eps[m] * np.sin((m + 1) * K1 * pos[0] + th[m]) for m in range(4))
            dt, steps, tol = 0.1, 200, 1e-10
            desc = "cold two-stream 32^3, 32 ppc/beam, quadratic, random 1e-3 over 4 kx modes"
        else:
            pert = sum(1e-3 * np.sin((m + 1) * K1 * pos[0]) for m in range(8))
            dt, steps, tol = 0.1, 50, 1e-13
            desc = "adjoint workload 32^3, 32 ppc/beam, quadratic, 1e-3 on 8 kx modes"
        r = 2
        prec = "fp64"
    elif name == "c4":
        n = (64, 64, 64)
        L = (LX, LX, LX)
        pos = _quiet_3d_lattice(n, L, 4)
        pert = None
        dt, steps, r, tol = 0.2, 100, 2, 1e-8
        prec = "mixed"
        desc = "two-stream 64^3, 4^3 lattice/cell/beam, quadratic, thermal 0.01"
    else:
        raise KeyError(name)
    if mesh is not None:
        mesh = tuple(int(k) for k in mesh)
        if name != "c4" and mesh[0] != n[0]:
            raise ValueError(f"{name}: the perturbation needs the x extent of {n[0]} cells")
        H = L[0] / n[0]
        n = mesh
        L = tuple(k * H for k in mesh)
        pos = _quiet_3d_lattice(n, L, 4) if name == "c4" else _quiet_x_lattice(n, L, ppb)
        if name == "c2":
            pert = sum(eps[m] * np.sin((m + 1) * K1 * pos[0] + th[m]) for m in range(4))
        elif name == "c5":
            pert = sum(1e-3 * np.sin((m + 1) * K1 * pos[0]) for m in range(8))
        elif name in ("c1", "c3"):
            pert = 1e-3 * np.sin(K1 * pos[0])
        desc = desc + " on a {}x{}x{} mesh".format(*mesh)

    k = pos.shape[1] // int(np.prod(n))  # points per cell per beam
    ncell = int(np.prod(n))
    # per cell: beam + block then beam - block (cell-major ordering)
    p3 = pos.reshape(3, ncell, 1, k)
    p3 = np.broadcast_to(p3, (3, ncell, 2, k))
    x = np.ascontiguousarray(p3.reshape(3, -1))
    sign = np.broadcast_to(np.array([1.0, -1.0]).reshape(1, 2, 1), (ncell, 2, k)).reshape(-1)
    v = np.zeros_like(x)
    if pert is not None:
        pr = np.broadcast_to(pert.reshape(ncell, 1, k), (ncell, 2, k)).reshape(-1)
        v[0] = sign * V0 + pr
    else:
        v[0] = sign * V0
        v += rng.normal(0.0, 0.01, size=v.shape)
    q, m = _species(1.0, L, x.shape[1])
    return Workload(name=name, n=n, L=L, dt=dt, steps=steps, r=r, tol=tol, pmax=16,
                    precision=prec, x=x, v=v, q=q, m=m, description=desc)


def paper_two_stream(steps: int = 1200) -> Workload:
    """The paper's own demonstration run (Sec. 5.4): 16^3 mesh on
    [0, 2 pi]^3, 16 particles per cell per beam on the cell-centred x lattice
    with both beams at identical positions (131,072 particles), drift
    v0 = 0.3, v_x = +-v0 + 0.02 sin(x) on both beams (k = 2 pi m / L_x, m = 1),
    v_y = v_z = 0, linear shape, dt = 0.025 for 1200 steps (T = 30), Picard
    tolerance 1e-11 and p_max = 16.  The paper's Gauss rule has 16 points per
    piece (identical to the closed forms when the orbit is split)."""
    n = (16, 16, 16)
    L = (2.0 * math.pi,) * 3
    k = 16
    pos = _quiet_x_lattice(n, L, k)
    ncell = int(np.prod(n))
    p3 = np.broadcast_to(pos.reshape(3, ncell, 1, k), (3, ncell, 2, k))
    x = np.ascontiguousarray(p3.reshape(3, -1))
    sign = np.broadcast_to(np.array([1.0, -1.0]).reshape(1, 2, 1), (ncell, 2, k)).reshape(-1)
    v = np.zeros_like(x)
    v[0] = sign * 0.3 + 0.02 * np.sin(x[0])
    q, m = _species(1.0, L, x.shape[1])
    return Workload(name="paper", n=n, L=L, dt=0.025, steps=steps, r=1, tol=1e-11, pmax=16,
                    precision="fp64", x=x, v=v, q=q, m=m,
                    description="paper's cold two-stream 16^3, L = 2 pi, v0 = 0.3, 131072 particles")


def random_plasma(n, L, np_, r, dt, vth, drift=(0.0, 0.0, 0.0), seed=SEED, tol=1e-12,
                  pmax=16, name="random") -> Workload:
    """Uniform random positions and Maxwellian velocities (for parity cases
    whose orbits cross knots along every axis).  Not cell-sorted."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.stack([rng.uniform(0.0, L[a], size=np_) for a in range(3)])
    v = rng.normal(0.0, vth, size=(3, np_)) + np.asarray(drift, dtype=float).reshape(3, 1)
    q, m = _species(1.0, L, np_)
    return Workload(name=name, n=tuple(n), L=tuple(L), dt=dt, steps=1, r=r, tol=tol, pmax=pmax,
                    precision="fp64", x=x, v=v, q=q, m=m, description="random plasma")


def electron_ion(n, L, np_, r, dt, vth, mass_ratio=16.0, drift=(0.0, 0.0, 0.0), seed=SEED,
                 tol=1e-12, pmax=16) -> Workload:
    """Neutral electron-ion plasma: np_ // 2 electrons (q/m = -1, uniform
    random positions, Maxwellian velocities of spread vth plus drift) and as
    many ions of charge +|q_e| and mass mass_ratio m_e at the electrons'
    positions, with spread vth / sqrt(mass_ratio) and no drift.  No background
    charge (n0 = 0); species 0 = electrons, 1 = ions, interleaved."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ne = np_ // 2
    xe = np.stack([rng.uniform(0.0, L[a], size=ne) for a in range(3)])
    ve = rng.normal(0.0, vth, size=(3, ne)) + np.asarray(drift, dtype=float).reshape(3, 1)
    vi = rng.normal(0.0, vth / math.sqrt(mass_ratio), size=(3, ne))
    x = np.empty((3, 2 * ne))
    v = np.empty((3, 2 * ne))
    x[:, 0::2], x[:, 1::2] = xe, xe
    v[:, 0::2], v[:, 1::2] = ve, vi
    species = np.tile(np.array([0, 1], dtype=np.int32), ne)
    qe, me = _species(1.0, L, ne)
    qs, ms = (qe, -qe), (me, mass_ratio * me)
    return Workload(name="electron-ion", n=tuple(n), L=tuple(L), dt=dt, steps=1, r=r, tol=tol,
                    pmax=pmax, precision="fp64", x=x, v=v, q=qe, m=me, n0=0.0,
                    description=f"electron-ion plasma, mass ratio {mass_ratio:g}",
                    species=species, qs=qs, ms=ms)


def plasma_oscillation(mass_ratio, r=1, dt=0.05, amp=1e-4) -> Workload:
    """Cold electron-ion plasma on the 16x4x4 two-stream box: 8 electrons and
    8 ions per cell at the same quiet x-lattice positions (rho^0 = 0), ions at
    rest, electrons with v_x = amp sin(k1 x); Langmuir oscillation of the k1
    mode."""
    n = (16, 4, 4)
    L = (LX, LX / 4, LX / 4)
    pos = _quiet_x_lattice(n, L, 8)
    ne = pos.shape[1]
    x = np.concatenate([pos, pos], axis=1)
    v = np.zeros_like(x)
    v[0, :ne] = amp * np.sin(K1 * pos[0])
    species = np.r_[np.zeros(ne, np.int32), np.ones(ne, np.int32)]
    qe, me = _species(1.0, L, ne)
    return Workload(name="plasma-oscillation", n=n, L=L, dt=dt, steps=500, r=r, tol=1e-13,
                    pmax=30, precision="fp64", x=x, v=v, q=qe, m=me, n0=0.0,
                    description=f"cold electron-ion Langmuir oscillation, mass ratio {mass_ratio:g}",
                    species=species, qs=(qe, -qe), ms=(me, mass_ratio * me))


def random_fields(n, ncomp, seed=SEED, modes=3, scale=1.0):
    """Smooth random periodic mesh fields: a few low Fourier modes per component
    (real-space, shape (ncomp,) + n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = np.meshgrid(*[np.arange(n[a]) / n[a] for a in range(3)], indexing="ij")
    out = np.zeros((ncomp,) + tuple(n))
    for c in range(ncomp):
        out[c] += scale * rng.normal()
        for _ in range(modes):
            k = [int(rng.integers(-2, 3)) for _ in range(3)]
            ph = rng.uniform(0, 2 * math.pi)
            amp = scale * rng.normal()
            out[c] += amp * np.cos(2 * math.pi * (k[0] * g[0] + k[1] * g[1] + k[2] * g[2]) + ph)
    return out
