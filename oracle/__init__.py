"""Plain serial FP64 CPU oracle of the energy-conserving potential PIC step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(the HIP library under ``paper_2606_15035_amd``) never imports it, and the two
share no code.

The arithmetic lives in ``ecpic_oracle.c`` (built with gcc, no fast-math, no
FMA contraction); this module only marshals numpy arrays through ctypes.  Each
C function cites the passage of the paper (Christlieb, Chacon, Gong, "An
Energy-Conserving Unstaggered Electromagnetic-Potential Particle-in-Cell
Method, Part I") that it follows.

Array conventions (both here and in the C file):
  particles  component-major, shape (3, np): x[a, i]
  fields     real-space node arrays, node (ix, iy, iz) at flat index
             (ix * Ny + iy) * Nz + iz, i.e. numpy shape (Nx, Ny, Nz)
  state      fields stacked as [phi, psi, Ax, Ay, Az, Ux, Uy, Uz, rho]
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ecpic_oracle.c")
# ECPIC_ORACLE_SANITIZE=1: a separate build with AddressSanitizer and
# UndefinedBehaviorSanitizer (load it with libasan preloaded into python)
_SANITIZE = os.environ.get("ECPIC_ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "libecpic_oracle_san.so" if _SANITIZE else "libecpic_oracle.so")

GCC_CMD = (["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-Wall", "-shared", "-fPIC",
            "-ffp-contract=off", "-fno-fast-math"]
           + (["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all"] if _SANITIZE else [])
           + [_SRC, "-o", _LIB, "-lm"])


def build() -> str:
    """Compile the oracle shared library (always recompiles)."""
    subprocess.run(GCC_CMD, check=True)
    return _LIB


class Cfg(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("L", C.c_double * 3), ("kappa", C.c_double),
                ("sigma1", C.c_double), ("sigma2", C.c_double), ("dt", C.c_double),
                ("r", C.c_int32), ("split", C.c_int32), ("nq", C.c_int32),
                ("analytic", C.c_int32), ("tol", C.c_double), ("pmax", C.c_int32),
                ("anderson", C.c_int32)]


class StepInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("err_v", C.c_double),
                ("err_J", C.c_double)]


class Energy(C.Structure):
    _fields_ = [(k, C.c_double) for k in (
        "K", "W", "E_total", "R_field", "R_particle", "R_total", "gauge_max", "gauge_l2",
        "gauss_max", "gauss_l2", "RA_rms", "RA_max", "pou_max", "JE_mesh", "work_particle")]
    _fields_ = _fields_ + [("step", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        D = C.POINTER(C.c_double)
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(Cfg), C.c_int64]
        L.orc_destroy.argtypes = [P]
        L.orc_check_config.argtypes = [C.POINTER(Cfg)]
        L.orc_init_particles.argtypes = [P, D, D, C.c_double, C.c_double, C.c_double]
        L.orc_picard_step.argtypes = [P, C.POINTER(StepInfo)]
        L.orc_energy_diagnostics.argtypes = [P, C.POINTER(Energy)]
        L.orc_get_state.argtypes = [P, D, D, D, D, D]
        L.orc_set_state.argtypes = [P, D, D, D, D, D, C.c_double, C.c_double]
        L.orc_get_current.argtypes = [P, D]
        L.orc_field_solve.argtypes = [P, D]
        L.orc_field_energy_of.argtypes = [P, D, D, D]
        L.orc_field_energy_of.restype = C.c_double
        L.orc_orbit_gather.argtypes = [P, C.c_int64, D, D, D, D, D, D, D]
        L.orc_orbit_deposit.argtypes = [P, C.c_int64, D, D, D, D]
        L.orc_interp.argtypes = [P, C.c_int64, D, D, C.c_int, D]
        L.orc_breakpoints.argtypes = [P, D, D, D]
        L.orc_dft3.argtypes = [P, D, C.c_int]
        L.orc_ktilde.argtypes = [P, D]
        L.orc_gauss_rule.argtypes = [P, D, D]
        L.orc_gauss_legendre.argtypes = [C.c_int, D, D]
        L.orc_adjoint_step.argtypes = [P, D, D, D, D, D, D, D, D, D, D, C.c_double, C.c_int,
                                       C.POINTER(C.c_int)]
        L.orc_rebuild_P.argtypes = [P]
        L.orc_field_energy_grad.argtypes = [P, D]
        L.orc_set_trace.argtypes = [P, D, D, C.c_int]
        L.orc_init_species.argtypes = [P, D, D, C.POINTER(C.c_int32), C.c_int, D, D, C.c_double]
        L.orc_anderson_mix.argtypes = [C.c_int, C.c_int64, C.POINTER(D), C.POINTER(D), D, D]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_cfg(n, L, dt, r=1, kappa=1.0, sigma1=1.0, sigma2=1.0, split=True, nq=0,
             analytic=True, tol=1e-12, pmax=16, anderson=0) -> Cfg:
    c = Cfg()
    for a in range(3):
        c.n[a] = int(n[a])
        c.L[a] = float(L[a])
    c.kappa, c.sigma1, c.sigma2, c.dt = kappa, sigma1, sigma2, dt
    c.r, c.split, c.nq, c.analytic = int(r), int(bool(split)), int(nq), int(bool(analytic))
    c.tol, c.pmax = float(tol), int(pmax)
    c.anderson = int(anderson)
    return c


def anderson_mix(w_hist, g_hist):
    """One Anderson update from iterates w_hist[j] and images g_hist[j]
    (j = 0 newest; len = mk + 1).  Returns (w_next, gamma)."""
    mk = len(w_hist) - 1
    w = [_f64(a).ravel() for a in w_hist]
    g = [_f64(a).ravel() for a in g_hist]
    n = w[0].size
    PD = C.POINTER(C.c_double)
    wa = (PD * (mk + 1))(*[_p(a) for a in w])
    ga = (PD * (mk + 1))(*[_p(a) for a in g])
    out = np.zeros(n)
    gamma = np.zeros(max(mk, 1))
    if lib().orc_anderson_mix(mk, n, wa, ga, _p(out), _p(gamma)) != 0:
        raise ValueError("bad Anderson arguments")
    return out, gamma[:mk]


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    if lib().orc_gauss_legendre(int(n), _p(x), _p(w)) != 0:
        raise ValueError("n out of range")
    return x, w


class OracleSim:
    """Owner of one oracle simulation (host memory only)."""

    def __init__(self, cfg: Cfg, np_: int):
        self.cfg = cfg
        self.np = int(np_)
        self.n = tuple(cfg.n)
        self.ncell = int(np.prod(self.n))
        h = lib().orc_create(C.byref(cfg), self.np)
        if not h:
            raise ValueError("invalid oracle configuration")
        self._h = h
        self.q = None
        self.m = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    # -- state ------------------------------------------------------------
    def init_particles(self, x, v, q, m, n0):
        x = _f64(x).reshape(3, self.np)
        v = _f64(v).reshape(3, self.np)
        self.q, self.m = float(q), float(m)
        rc = lib().orc_init_particles(self._h, _p(x), _p(v), q, m, n0)
        if rc != 0:
            raise RuntimeError("orc_init_particles failed")

    def init_species(self, x, v, species, q, m, n0):
        """Several species: particle i has charge q[species[i]], mass m[species[i]]."""
        x = _f64(x).reshape(3, self.np)
        v = _f64(v).reshape(3, self.np)
        sp = np.ascontiguousarray(species, dtype=np.int32)
        q, m = _f64(q), _f64(m)
        self.q, self.m = float(q[0]), float(m[0])
        rc = lib().orc_init_species(self._h, _p(x), _p(v),
                                    sp.ctypes.data_as(C.POINTER(C.c_int32)), len(q), _p(q),
                                    _p(m), n0)
        if rc != 0:
            raise ValueError("orc_init_species: bad species")

    def step(self):
        info = StepInfo()
        rc = lib().orc_picard_step(self._h, C.byref(info))
        if rc < 0:
            raise RuntimeError("orc_picard_step failed")
        return {"iters": info.iters, "converged": bool(info.converged), "err_v": info.err_v,
                "err_J": info.err_J, "status": rc}

    def energy(self):
        e = Energy()
        lib().orc_energy_diagnostics(self._h, C.byref(e))
        return e.as_dict()

    def get_state(self):
        x = np.zeros((3, self.np))
        v = np.zeros((3, self.np))
        vp = np.zeros((3, self.np))
        P = np.zeros((3, self.np))
        f = np.zeros((9,) + self.n)
        lib().orc_get_state(self._h, _p(x), _p(v), _p(vp), _p(P), _p(f))
        return {"x": x, "v": v, "vprev": vp, "P": P, "fields": f}

    def set_state(self, x, v, vprev, P, fields, q, m):
        args = [None if a is None else _f64(a) for a in (x, v, vprev, P, fields)]
        self.q, self.m = float(q), float(m)
        lib().orc_set_state(self._h, *[_p(a) for a in args], q, m)

    def trace_next_step(self, max_passes):
        """Record the iterates and images of the passes of the next step.
        Returns (w, g) arrays of shape (max_passes, 3, np), filled by step()."""
        self._trace = (np.zeros((max_passes, 3, self.np)), np.zeros((max_passes, 3, self.np)))
        lib().orc_set_trace(self._h, _p(self._trace[0]), _p(self._trace[1]), int(max_passes))
        return self._trace

    def stop_trace(self):
        lib().orc_set_trace(self._h, None, None, 0)
        self._trace = None

    def current(self):
        J = np.zeros((3,) + self.n)
        lib().orc_get_current(self._h, _p(J))
        return J

    def field_solve(self, J):
        J = _f64(J).reshape((3,) + self.n)
        lib().orc_field_solve(self._h, _p(J))

    # -- adjoint ----------------------------------------------------------
    def rebuild_P(self):
        """P^n = m v^n + q A_h^n(x^n) from the present state."""
        lib().orc_rebuild_P(self._h)

    def field_energy_grad(self):
        """dW/dF for the present real-space fields, shape (9,) + n."""
        g = np.zeros((9,) + self.n)
        lib().orc_field_energy_grad(self._h, _p(g))
        return g

    def adjoint_step(self, x, v, w, F, lx1=None, lv1=None, lF1=None, tol=1e-14, maxit=200):
        """Adjoint of the converged step from (x, v, F) whose solution is w.
        Returns (lx0, lv0, lF0, iterations)."""
        x, v, w = (_f64(a).reshape(3, self.np) for a in (x, v, w))
        F = _f64(F).reshape((9,) + self.n)
        lx1, lv1 = (None if a is None else _f64(a).reshape(3, self.np) for a in (lx1, lv1))
        lF1 = None if lF1 is None else _f64(lF1).reshape((9,) + self.n)
        lx0 = np.zeros((3, self.np))
        lv0 = np.zeros((3, self.np))
        lF0 = np.zeros((9,) + self.n)
        it = C.c_int(0)
        rc = lib().orc_adjoint_step(self._h, _p(x), _p(v), _p(w), _p(F), _p(lx1), _p(lv1),
                                    _p(lF1), _p(lx0), _p(lv0), _p(lF0), float(tol), int(maxit),
                                    C.byref(it))
        if rc < 0:
            raise RuntimeError("orc_adjoint_step: degree 2 with split orbits only")
        if rc > 0:
            raise RuntimeError("orc_adjoint_step: transposed iteration did not converge")
        return lx0, lv0, lF0, it.value

    # -- kernel-level helpers (tests) -------------------------------------
    def field_energy_of(self, phi, A, U):
        return lib().orc_field_energy_of(self._h, _p(_f64(phi)), _p(_f64(A)), _p(_f64(U)))

    def orbit_gather(self, x0, d, gphi, Uh, A0, A1):
        """Per-particle orbit integrals; x0, d of shape (n, 3).  Returns dict."""
        x0 = _f64(x0).reshape(-1, 3)
        d = _f64(d).reshape(-1, 3)
        n = x0.shape[0]
        out = np.zeros((n, 24))
        fs = [_f64(f).reshape((3,) + self.n) for f in (gphi, Uh, A0, A1)]
        rc = lib().orc_orbit_gather(self._h, n, _p(x0), _p(d), *[_p(f) for f in fs], _p(out))
        if rc != 0:
            raise RuntimeError("orbit too long")
        return {"gphibar": out[:, 0:3], "Ubar": out[:, 3:6], "D": out[:, 6:15].reshape(n, 3, 3),
                "A1_end": out[:, 15:18], "A0_start": out[:, 18:21], "pou": out[:, 21],
                "npieces": out[:, 22].astype(int)}

    def orbit_deposit(self, x0, d, qv, J=None):
        x0 = _f64(x0).reshape(-1, 3)
        d = _f64(d).reshape(-1, 3)
        qv = _f64(qv).reshape(-1, 3)
        if J is None:
            J = np.zeros((3,) + self.n)
        rc = lib().orc_orbit_deposit(self._h, x0.shape[0], _p(x0), _p(d), _p(qv), _p(J))
        if rc != 0:
            raise RuntimeError("orbit too long")
        return J

    def interp(self, x, F):
        x = _f64(x).reshape(-1, 3)
        F = _f64(F)
        ncomp = F.size // self.ncell
        out = np.zeros((x.shape[0], ncomp))
        lib().orc_interp(self._h, x.shape[0], _p(x), _p(F), ncomp, _p(out))
        return out

    def breakpoints(self, x0, d):
        s = np.zeros(512)
        k = lib().orc_breakpoints(self._h, _p(_f64(x0)), _p(_f64(d)), _p(s))
        return s[:k].copy()

    def dft3(self, f, sign):
        a = np.ascontiguousarray(f, dtype=np.complex128).copy()
        lib().orc_dft3(self._h, a.view(np.float64).ctypes.data_as(C.POINTER(C.c_double)), sign)
        return a

    def ktilde(self):
        k = np.zeros((3,) + self.n)
        lib().orc_ktilde(self._h, _p(k))
        return k

    def gauss_rule(self):
        x = np.zeros(64)
        w = np.zeros(64)
        k = lib().orc_gauss_rule(self._h, _p(x), _p(w))
        return x[:k].copy(), w[:k].copy()
