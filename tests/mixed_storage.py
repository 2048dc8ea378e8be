"""What the mixed-precision particle storage holds, computed on the host, and
the one-step comparison of a mixed GPU step with the FP64 oracle.

The mixed form stores a position as its cell and an FP32 offset inside the
cell (in cell units) and a velocity as FP32.  A parity case starts both sides
from a state that this storage represents exactly; within the step they then
differ only by the current's quantisation (at most half a quantum,
2^-41 |q| / dV, per contribution), and at the end the GPU rounds its accepted
state to the storage format, so its stored state equals the oracle's result
rounded the same way to one FP32 unit in the last place.
"""
import numpy as np


def to_storage(wl, x, v):
    """The values the mixed storage holds for positions x and velocities v:
    x = (c + f) H with c = floor(x / H) and f = x / H - c rounded to FP32
    (an offset that rounds up to 1 moves to the next cell), v rounded to FP32."""
    H = (np.asarray(wl.L) / np.asarray(wl.n)).reshape(3, 1)
    n = np.asarray(wl.n).reshape(3, 1)
    Lr = np.asarray(wl.L).reshape(3, 1)
    xw = x - Lr * np.floor(x / Lr)
    u = xw / H
    c = np.floor(u)
    f = (u - c).astype(np.float32).astype(np.float64)
    up = f >= 1.0
    f[up] = 0.0
    c[up] += 1.0
    c = np.mod(c, n)
    return (c + f) * H, v.astype(np.float32).astype(np.float64)


def ulp32(a):
    return np.spacing(np.abs(a).astype(np.float32)).astype(np.float64)


def check_mixed_step(wl, x0, v0, sg, so, Jg, Jo, log, name, pieces=2):
    """Stored GPU state sg against the oracle's so after one step from the
    storage-exact (x0, v0); Jg, Jo the two orbit currents; pieces: most orbit
    pieces of one particle in the step (sets the current bound)."""
    xe, ve = to_storage(wl, so["x"], so["v"])
    H = (np.asarray(wl.L) / np.asarray(wl.n)).reshape(3, 1)
    dx = np.abs(sg["x"] - xe)
    dx = np.minimum(dx, np.abs(dx - np.asarray(wl.L).reshape(3, 1)))  # periodic images
    dv = np.abs(sg["v"] - ve)
    # one FP32 ulp of the value, plus the FP64 parity level for components
    # that are roundoff-sized (e.g. v_y of a beam along x)
    vtol = ulp32(ve) * 1.0000001 + 1e-12 * np.abs(so["v"]).max()
    log(f"[{name}] max|dx|/H = {np.max(dx / H):.2e}  max|dv|/tol = {np.max(dv / vtol):.2f}")
    assert np.all(dx <= 2.0 ** -24 * H * 1.0000001 + 1e-12 * np.abs(so["v"]).max() * wl.dt)
    assert np.all(dv <= vtol)
    assert np.array_equal(sg["vprev"], v0)  # v^{n-1} <- v^n, stored exactly
    # the current: at most half a quantum per contribution; a node collects
    # (r+1)^3 contributions per particle piece from the cells around it
    dV = np.prod(H)
    ppn = wl.np / np.prod(wl.n)
    bound = (wl.r + 1) ** 3 * ppn * pieces * 2.0 ** -41 * abs(wl.q) / dV
    errJ = np.abs(Jg - Jo).max()
    log(f"[{name}] max|dJ| = {errJ:.2e} (bound {bound:.2e})")
    assert errJ <= bound
    # fields: FP64 CN solve from the quantised current.  A current error dJ
    # moves rho by at most dt |k| dJ (|k| <= sqrt(3) pi / H) and the
    # potentials by less than dt dJ L; these set the tolerance next to the
    # FP64 parity level.
    dfield = wl.dt * bound * (np.sqrt(3.0) * np.pi / H.min() + max(wl.L))
    for nm, ks in (("phi", [0]), ("psi", [1]), ("A", [2, 3, 4]), ("U", [5, 6, 7]), ("rho", [8])):
        ref = so["fields"][ks]
        scale = max(np.abs(ref).max(), 1e-300)
        err = np.abs(sg["fields"][ks] - ref).max()
        log(f"[{name}] {nm}: max err {err:.2e}, scale {scale:.2e}, current-induced {dfield:.2e}")
        assert err <= 1e-10 * scale + dfield, (nm, err, scale)
