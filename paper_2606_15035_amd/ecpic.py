"""Thin Python binding of the C ABI in include/ecpic.h (libecpic.so).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch provides the device memory (the caller-owned state
and workspace buffers) and the HIP stream.  If the library is not built, or
no GPU is visible, the binding raises; there is no CPU fallback.

Function names follow the C ABI: ``state_bytes``, ``Sim.init_particles``,
``Sim.picard_step``, ``Sim.field_solve``, ``Sim.energy_diagnostics``,
``Sim.get_state``, ``Sim.set_state``, ``Sim.get_current``, ``orbit_gather``,
``orbit_deposit``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libecpic.so")

OK, ENOCONV, EINVAL, ENOMEM, EDEVICE, ENONFINITE, ESTATE = 0, 1, -1, -2, -3, -4, -5
FP64, MIXED = 0, 1


class EcpicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ecpic status {status}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("spline_degree", C.c_int32), ("L", C.c_double * 3),
                ("kappa", C.c_double), ("sigma1", C.c_double), ("sigma2", C.c_double),
                ("dt", C.c_double), ("picard_tol", C.c_double), ("picard_max", C.c_int32),
                ("split_orbit_at_knots", C.c_int32), ("quad_points", C.c_int32),
                ("precision", C.c_int32), ("fixed_point_scale", C.c_double),
                ("diagnostics", C.c_int32), ("sort_interval", C.c_int32),
                ("anderson_depth", C.c_int32), ("scatter_chunk", C.c_int32)]


class StepInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("err_v", C.c_double),
                ("err_J", C.c_double)]


_ENERGY_FIELDS = ("K", "W", "E_total", "R_field", "R_particle", "R_total", "gauge_max",
                  "gauge_l2", "gauss_max", "gauss_l2", "RA_rms", "RA_max", "pou_max", "JE_mesh",
                  "work_particle")


class Energy(C.Structure):
    _fields_ = [(k, C.c_double) for k in _ENERGY_FIELDS] + [("step", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Profile(C.Structure):
    _fields_ = [("ms", C.c_double * 8), ("launches", C.c_int64 * 8), ("pieces", C.c_double),
                ("scatter_chunk", C.c_int32), ("reserved", C.c_int32)]

    PHASES = ("scatter", "field_solve", "gather_push", "sweep", "finalize", "step")

    def as_dict(self):
        return {name: {"ms": self.ms[i], "launches": self.launches[i]}
                for i, name in enumerate(self.PHASES)} | {"pieces": self.pieces,
                                                           "scatter_chunk": self.scatter_chunk}


class AdjointInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("err", C.c_double)]


_lib = None


def lib():
    """Load libecpic.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2606_15035_amd.build")
        L = C.CDLL(LIB_PATH)
        P, D, I64 = C.c_void_p, C.c_void_p, C.c_int64
        cfgp = C.POINTER(Config)
        L.ecpic_state_bytes.argtypes = [cfgp, I64, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
        L.ecpic_create.argtypes = [cfgp, I64, P, C.c_size_t, P, C.c_size_t, P, C.POINTER(P)]
        L.ecpic_destroy.argtypes = [P]
        L.ecpic_destroy.restype = None
        L.ecpic_init_particles.argtypes = [P, D, D, C.c_double, C.c_double, C.c_double]
        L.ecpic_init_species.argtypes = [P, D, D, C.POINTER(C.c_int32), C.c_int32, D, D,
                                         C.c_double]
        L.ecpic_picard_step.argtypes = [P, C.POINTER(StepInfo)]
        L.ecpic_field_solve.argtypes = [P, D]
        L.ecpic_energy_diagnostics.argtypes = [P, C.POINTER(Energy)]
        L.ecpic_get_state.argtypes = [P, D, D, D, D]
        L.ecpic_set_state.argtypes = [P, D, D, D, D, C.c_double, C.c_double]
        L.ecpic_get_current.argtypes = [P, D]
        L.ecpic_orbit_gather.argtypes = [cfgp, I64, D, D, D, D, D, D, D, P]
        L.ecpic_orbit_deposit.argtypes = [cfgp, I64, D, D, D, D, P]
        L.ecpic_set_profiling.argtypes = [P, C.c_int32]
        L.ecpic_get_profile.argtypes = [P, C.POINTER(Profile)]
        L.ecpic_adjoint_workspace_bytes.argtypes = [cfgp, I64, C.POINTER(C.c_size_t)]
        L.ecpic_adjoint_step.argtypes = [P, P, C.c_size_t, D, D, D, D, D, D, D, D, D, D,
                                         C.c_double, C.c_int32, C.POINTER(AdjointInfo)]
        L.ecpic_adjoint_step_noalloc.argtypes = [P, D, D, D, D, D, D, D, D, D, D, C.c_double,
                                                 C.c_int32, C.POINTER(AdjointInfo)]
        L.ecpic_checkpoint_bytes.argtypes = [P, C.POINTER(C.c_size_t)]
        L.ecpic_checkpoint_save.argtypes = [P, P]
        L.ecpic_checkpoint_restore.argtypes = [P, P]
        L.ecpic_field_energy_grad.argtypes = [P, D]
        L.ecpic_measure_peaks.argtypes = [P, C.c_size_t, C.c_int32, P, C.POINTER(C.c_double),
                                          C.POINTER(C.c_double)]
        L.ecpic_last_error.restype = C.c_char_p
        L.ecpic_version.restype = C.c_char_p
        for name in ("ecpic_state_bytes", "ecpic_create", "ecpic_init_particles",
                     "ecpic_init_species",
                     "ecpic_picard_step", "ecpic_field_solve", "ecpic_energy_diagnostics",
                     "ecpic_get_state", "ecpic_set_state", "ecpic_get_current",
                     "ecpic_orbit_gather", "ecpic_orbit_deposit", "ecpic_set_profiling",
                     "ecpic_get_profile", "ecpic_adjoint_workspace_bytes",
                     "ecpic_adjoint_step", "ecpic_adjoint_step_noalloc",
                     "ecpic_checkpoint_bytes", "ecpic_checkpoint_save",
                     "ecpic_checkpoint_restore", "ecpic_field_energy_grad",
                     "ecpic_measure_peaks"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(status, allow=(OK,)):
    if status not in allow:
        raise EcpicError(status, lib().ecpic_last_error().decode())
    return status


def make_config(n, L, dt, r=1, kappa=1.0, sigma1=1.0, sigma2=1.0, tol=1e-12, pmax=16,
                split=True, quad_points=0, precision=FP64, fixed_point_scale=0.0,
                diagnostics=False, sort_interval=0, anderson=0, scatter_chunk=0) -> Config:
    c = Config()
    for a in range(3):
        c.n[a] = int(n[a])
        c.L[a] = float(L[a])
    c.spline_degree = int(r)
    c.kappa, c.sigma1, c.sigma2, c.dt = float(kappa), float(sigma1), float(sigma2), float(dt)
    c.picard_tol, c.picard_max = float(tol), int(pmax)
    c.split_orbit_at_knots = int(bool(split))
    c.quad_points = int(quad_points)
    c.precision = int(precision)
    c.fixed_point_scale = float(fixed_point_scale)
    c.diagnostics = int(bool(diagnostics))
    c.sort_interval = int(sort_interval)
    c.anderson_depth = int(anderson)
    c.scatter_chunk = int(scatter_chunk)
    return c


# bytes of the library's fixed workspace of ecpic_adjoint_step_noalloc
# (ECPIC_STATIC_SCRATCH_BYTES in include/ecpic.h)
STATIC_SCRATCH_BYTES = 64 << 20


def adjoint_workspace_bytes(cfg: Config, n_particles: int) -> int:
    nb = C.c_size_t()
    _check(lib().ecpic_adjoint_workspace_bytes(C.byref(cfg), int(n_particles), C.byref(nb)))
    return nb.value


def state_bytes(cfg: Config, n_particles: int):
    s, w = C.c_size_t(), C.c_size_t()
    _check(lib().ecpic_state_bytes(C.byref(cfg), int(n_particles), C.byref(s), C.byref(w)))
    return s.value, w.value


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the ecpic library needs a gfx950 device")
    return torch


def _host(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _hp(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Sim:
    """A simulation over torch-allocated device buffers on the current stream."""

    def __init__(self, cfg: Config, n_particles: int, device="cuda", stream=None):
        torch = _torch()
        self.torch = torch
        self.cfg = cfg
        self.np = int(n_particles)
        self.n = tuple(cfg.n)
        self.ncell = int(np.prod(self.n))
        sb, wb = state_bytes(cfg, self.np)
        self.state = torch.empty(sb, dtype=torch.uint8, device=device)
        self.workspace = torch.empty(wb, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.state.device)
        h = C.c_void_p()
        _check(lib().ecpic_create(C.byref(cfg), self.np, C.c_void_p(self.state.data_ptr()), sb,
                                  C.c_void_p(self.workspace.data_ptr()), wb,
                                  C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self.q = None
        self.m = None

    def close(self):
        if getattr(self, "_h", None):
            lib().ecpic_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_particles(self, x, v, q, m, n0=1.0):
        x = _host(x, (3, self.np))
        v = _host(v, (3, self.np))
        self.q, self.m = float(q), float(m)
        _check(lib().ecpic_init_particles(self._h, _hp(x), _hp(v), float(q), float(m), float(n0)))

    def init_species(self, x, v, species, q, m, n0=0.0):
        """Several species: particle i has charge q[species[i]], mass m[species[i]]."""
        x = _host(x, (3, self.np))
        v = _host(v, (3, self.np))
        sp = np.ascontiguousarray(species, dtype=np.int32).reshape(self.np)
        qa = np.ascontiguousarray(q, dtype=np.float64)
        ma = np.ascontiguousarray(m, dtype=np.float64)
        self.q, self.m = float(qa[0]), float(ma[0])
        _check(lib().ecpic_init_species(self._h, _hp(x), _hp(v),
                                        sp.ctypes.data_as(C.POINTER(C.c_int32)), len(qa),
                                        _hp(qa), _hp(ma), float(n0)))

    def picard_step(self):
        info = StepInfo()
        st = _check(lib().ecpic_picard_step(self._h, C.byref(info)), allow=(OK, ENOCONV))
        return {"iters": info.iters, "converged": bool(info.converged), "err_v": info.err_v,
                "err_J": info.err_J, "status": st}

    def field_solve(self, J_dev=None):
        ptr = None if J_dev is None else C.c_void_p(J_dev.data_ptr())
        _check(lib().ecpic_field_solve(self._h, ptr))

    def energy_diagnostics(self):
        e = Energy()
        _check(lib().ecpic_energy_diagnostics(self._h, C.byref(e)))
        return e.as_dict()

    def get_state(self, device=False):
        """x, v, v^{n-1} (3, np) in the caller's order and the real-space fields
        (9,) + n: host arrays, or with device=True float64 tensors on the
        simulation's device (no trip through host memory)."""
        shapes = {"x": (3, self.np), "v": (3, self.np), "vprev": (3, self.np),
                  "fields": (9,) + self.n}
        if device:
            torch = self.torch
            out = {k: torch.empty(sh, dtype=torch.float64, device=self.state.device)
                   for k, sh in shapes.items()}
            ptrs = [C.c_void_p(out[k].data_ptr()) for k in shapes]
        else:
            out = {k: np.zeros(sh) for k, sh in shapes.items()}
            ptrs = [_hp(out[k]) for k in shapes]
        _check(lib().ecpic_get_state(self._h, *ptrs))
        return out

    def get_fields(self):
        """Real-space mesh fields only (9,) + n: phi, psi, A, U, rho."""
        f = np.zeros((9,) + self.n)
        _check(lib().ecpic_get_state(self._h, None, None, None, _hp(f)))
        return f

    def set_state(self, x=None, v=None, vprev=None, fields=None, q=None, m=None):
        """Replace parts of the state.  With q and m every particle becomes of
        that one species; without them every particle keeps its species."""
        args = [self._any(a) for a in (x, v, vprev, fields)]  # host arrays or device tensors
        if m is None:
            q, m = 0.0, 0.0
        else:
            q, m = float(q), float(m)
            self.q, self.m = q, m
        _check(lib().ecpic_set_state(self._h, *[p for _, p in args], q, m))

    def _any(self, a):
        """(kept object, pointer) for a host array or a device tensor (float64,
        contiguous); (None, None) for None."""
        if a is None:
            return None, None
        torch = self.torch
        if isinstance(a, torch.Tensor) and a.is_cuda:
            t = a.to(dtype=torch.float64).contiguous()
            return t, C.c_void_p(t.data_ptr())
        h = _host(a)
        return h, _hp(h)

    def checkpoint(self) -> np.ndarray:
        """The simulation's state as a host byte array (ecpic_checkpoint_save)."""
        nb = C.c_size_t()
        _check(lib().ecpic_checkpoint_bytes(self._h, C.byref(nb)))
        buf = np.empty(nb.value, dtype=np.uint8)
        _check(lib().ecpic_checkpoint_save(self._h, buf.ctypes.data_as(C.c_void_p)))
        return buf

    def restore(self, buf: np.ndarray):
        """Continue from a checkpoint of a simulation of the same configuration."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib().ecpic_checkpoint_restore(self._h, buf.ctypes.data_as(C.c_void_p)))

    def set_profiling(self, level=1):
        """0 off, 1 (or True) every phase, 2 the gather phase only."""
        _check(lib().ecpic_set_profiling(self._h, int(level)))

    def get_profile(self):
        p = Profile()
        _check(lib().ecpic_get_profile(self._h, C.byref(p)))
        return p.as_dict()

    def get_current(self):
        J = np.zeros((3,) + self.n)
        _check(lib().ecpic_get_current(self._h, _hp(J)))
        return J

    # -- adjoint ----------------------------------------------------------
    def _dev(self, a, shape):
        """float64 contiguous device tensor of the given shape (or None)."""
        if a is None:
            return None
        torch = self.torch
        t = torch.as_tensor(a, dtype=torch.float64, device=self.state.device)
        return t.reshape(shape).contiguous()

    def field_energy_grad(self):
        """dW/dF of the present fields: device tensor (9,) + n."""
        torch = self.torch
        g = torch.empty((9,) + self.n, dtype=torch.float64, device=self.state.device)
        _check(lib().ecpic_field_energy_grad(self._h, C.c_void_p(g.data_ptr())))
        return g

    def adjoint_step(self, x, v, w, F, lx1=None, lv1=None, lF1=None, tol=1e-13, max_iters=100,
                     noalloc=False):
        """Adjoint of the converged step from (x, v, F) whose solution is w
        (arrays or tensors; particles in the caller's order).  Returns device
        tensors (lx0, lv0, lF0) and the iteration info.  noalloc: call
        ecpic_adjoint_step_noalloc (the library's own fixed workspace) instead
        of ecpic_adjoint_step with a workspace tensor."""
        torch = self.torch
        if not noalloc and getattr(self, "_adj_ws", None) is None:
            nb = C.c_size_t()
            _check(lib().ecpic_adjoint_workspace_bytes(C.byref(self.cfg), self.np, C.byref(nb)))
            self._adj_ws = torch.empty(nb.value, dtype=torch.uint8, device=self.state.device)
        p3, pf = (3, self.np), (9,) + self.n
        x, v, w, lx1, lv1 = (self._dev(a, p3) for a in (x, v, w, lx1, lv1))
        F, lF1 = self._dev(F, pf), self._dev(lF1, pf)
        lx0 = torch.empty(p3, dtype=torch.float64, device=self.state.device)
        lv0 = torch.empty(p3, dtype=torch.float64, device=self.state.device)
        lF0 = torch.empty(pf, dtype=torch.float64, device=self.state.device)
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())  # noqa: E731
        info = AdjointInfo()
        args = (ptr(x), ptr(v), ptr(w), ptr(F), ptr(lx1), ptr(lv1), ptr(lF1), ptr(lx0), ptr(lv0),
                ptr(lF0), float(tol), int(max_iters), C.byref(info))
        if noalloc:
            st = lib().ecpic_adjoint_step_noalloc(self._h, *args)
        else:
            st = lib().ecpic_adjoint_step(self._h, C.c_void_p(self._adj_ws.data_ptr()),
                                          self._adj_ws.numel(), *args)
        _check(st, allow=(OK, ENOCONV))
        return lx0, lv0, lF0, {"iters": info.iters, "converged": bool(info.converged),
                               "err": info.err}


def orbit_gather(cfg: Config, x0, d, gphi, U, A0, A1, device="cuda"):
    """Kernel-level orbit integrals of n particles; x0, d host arrays (n, 3);
    fields host arrays (3,) + n.  Returns a dict of host arrays."""
    torch = _torch()
    x0 = np.ascontiguousarray(np.asarray(x0, dtype=np.float64).reshape(-1, 3).T)
    d = np.ascontiguousarray(np.asarray(d, dtype=np.float64).reshape(-1, 3).T)
    n = x0.shape[1]
    t = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)
         for a in (x0, d, gphi, U, A0, A1)]
    out = torch.zeros((n, 24), dtype=torch.float64, device=device)
    s = torch.cuda.current_stream()
    _check(lib().ecpic_orbit_gather(C.byref(cfg), n, *[C.c_void_p(a.data_ptr()) for a in t],
                                    C.c_void_p(out.data_ptr()), C.c_void_p(s.cuda_stream)))
    o = out.cpu().numpy()
    return {"gphibar": o[:, 0:3], "Ubar": o[:, 3:6], "D": o[:, 6:15].reshape(n, 3, 3),
            "A1_end": o[:, 15:18], "A0_start": o[:, 18:21], "pou": o[:, 21],
            "npieces": o[:, 22].astype(int)}


def measure_peaks(nbytes=4 << 30, repeats=5):
    """Measured FP64 TFLOP/s and HBM GB/s of the current device
    (ecpic_measure_peaks) over a device buffer of nbytes."""
    torch = _torch()
    buf = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
    f, h = C.c_double(), C.c_double()
    s = torch.cuda.current_stream()
    _check(lib().ecpic_measure_peaks(C.c_void_p(buf.data_ptr()), int(nbytes), int(repeats),
                                     C.c_void_p(s.cuda_stream), C.byref(f), C.byref(h)))
    del buf
    return {"fp64_tflops": f.value, "hbm_GBs": h.value}


def orbit_deposit(cfg: Config, x0, d, qv, device="cuda"):
    torch = _torch()
    x0 = np.ascontiguousarray(np.asarray(x0, dtype=np.float64).reshape(-1, 3).T)
    d = np.ascontiguousarray(np.asarray(d, dtype=np.float64).reshape(-1, 3).T)
    qv = np.ascontiguousarray(np.asarray(qv, dtype=np.float64).reshape(-1, 3).T)
    n = x0.shape[1]
    t = [torch.from_numpy(a).to(device) for a in (x0, d, qv)]
    ncell = int(np.prod(tuple(cfg.n)))
    J = torch.zeros(3 * ncell, dtype=torch.float64, device=device)
    s = torch.cuda.current_stream()
    _check(lib().ecpic_orbit_deposit(C.byref(cfg), n, *[C.c_void_p(a.data_ptr()) for a in t],
                                     C.c_void_p(J.data_ptr()), C.c_void_p(s.cuda_stream)))
    return J.cpu().numpy().reshape((3,) + tuple(cfg.n))
