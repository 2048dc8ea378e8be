"""Brute-force references used to pin the CPU oracle.

Nothing here is shared with the oracle or the HIP path.  The B-splines are
written from their textbook definition (centred cardinal B-spline of degree r),
knot crossings of an orbit are located by bisection on the polynomial-piece
index, and orbit integrals are evaluated with numpy's Gauss-Legendre rule
(``numpy.polynomial.legendre.leggauss``) on every knot-free piece.  Everything
is slow and only meant for a handful of particles.
"""
from __future__ import annotations

import math

import numpy as np


def M(r: int, xi: float) -> float:
    """Centred cardinal B-spline of degree r (1: hat, 2: quadratic, 3: cubic)."""
    a = abs(xi)
    if r == 1:
        return max(0.0, 1.0 - a)
    if r == 2:
        if a <= 0.5:
            return 0.75 - a * a
        if a <= 1.5:
            return 0.5 * (1.5 - a) ** 2
        return 0.0
    if r == 3:
        if a <= 1.0:
            return 2.0 / 3.0 - a * a + 0.5 * a ** 3
        if a <= 2.0:
            return (2.0 - a) ** 3 / 6.0
        return 0.0
    raise ValueError(r)


def dM(r: int, xi: float) -> float:
    """Derivative of M (one-sided value is irrelevant under an integral)."""
    a = abs(xi)
    s = 1.0 if xi > 0 else -1.0
    if r == 1:
        return -s if a < 1.0 else 0.0
    if r == 2:
        if a <= 0.5:
            return -2.0 * xi
        if a <= 1.5:
            return -s * (1.5 - a)
        return 0.0
    if r == 3:
        if a <= 1.0:
            return s * (-2.0 * a + 1.5 * a * a)
        if a <= 2.0:
            return -s * 0.5 * (2.0 - a) ** 2
        return 0.0
    raise ValueError(r)


def _axis_nodes(r, u, N):
    """(wrapped node, unwrapped distance u - g) of the nodes whose B-spline
    covers u, found by scanning a generous neighbourhood."""
    base = math.floor(u)
    out = []
    for g in range(base - 3, base + 4):
        xi = u - g
        if abs(xi) < (r + 1) / 2.0:
            out.append((g % N, xi))
    return out


def point_values(r, x, n, L, F, deriv=False):
    """sum_g F_g S_g(x) (and its gradient when deriv) for F of shape (c,)+n."""
    H = [L[a] / n[a] for a in range(3)]
    u = [x[a] / H[a] for a in range(3)]
    nodes = [_axis_nodes(r, u[a], n[a]) for a in range(3)]
    val = np.zeros(F.shape[0])
    grad = np.zeros((F.shape[0], 3))
    for gx, xx in nodes[0]:
        for gy, xy in nodes[1]:
            for gz, xz in nodes[2]:
                w = (M(r, xx), M(r, xy), M(r, xz))
                f = F[:, gx, gy, gz]
                val += f * (w[0] * w[1] * w[2])
                if deriv:
                    dw = (dM(r, xx) / H[0], dM(r, xy) / H[1], dM(r, xz) / H[2])
                    grad[:, 0] += f * dw[0] * w[1] * w[2]
                    grad[:, 1] += f * w[0] * dw[1] * w[2]
                    grad[:, 2] += f * w[0] * w[1] * dw[2]
    return (val, grad) if deriv else val


def shape_weights(r, x, n, L):
    """{(gx, gy, gz): S_g(x)} for the nodes whose shape covers x."""
    H = [L[a] / n[a] for a in range(3)]
    nodes = [_axis_nodes(r, x[a] / H[a], n[a]) for a in range(3)]
    out = {}
    for gx, xx in nodes[0]:
        for gy, xy in nodes[1]:
            for gz, xz in nodes[2]:
                w = M(r, xx) * M(r, xy) * M(r, xz)
                if w != 0.0:
                    out[(gx, gy, gz)] = out.get((gx, gy, gz), 0.0) + w
    return out


def knot_crossings(r, x0, d, n, L, scan=4000):
    """Orbit parameters s in (0,1) where x0 + s d crosses a spline knot, found by
    bisection on the index of the polynomial piece (knots at integers for the
    hat and the cubic spline, at half-integers for the quadratic spline)."""
    off = 0.5 if r == 2 else 0.0
    out = []
    for a in range(3):
        if d[a] == 0.0:
            continue
        H = L[a] / n[a]

        def piece(s):
            return math.floor((x0[a] + s * d[a]) / H - off)

        ss = np.linspace(0.0, 1.0, scan + 1)
        ks = [piece(s) for s in ss]
        for i in range(scan):
            if ks[i] != ks[i + 1]:
                lo, hi = ss[i], ss[i + 1]
                klo = ks[i]
                for _ in range(200):
                    mid = 0.5 * (lo + hi)
                    if piece(mid) == klo:
                        lo = mid
                    else:
                        hi = mid
                    if hi - lo < 1e-17:
                        break
                out.append(0.5 * (lo + hi))
    return sorted(out)


def orbit_integral(f, r, x0, d, n, L, order=12):
    """int_0^1 f(s) ds for an integrand that is polynomial between knot
    crossings: Gauss-Legendre of the given order on every piece."""
    cuts = [0.0] + [s for s in knot_crossings(r, x0, d, n, L) if 0.0 < s < 1.0] + [1.0]
    gx, gw = np.polynomial.legendre.leggauss(order)
    total = None
    for a, b in zip(cuts[:-1], cuts[1:]):
        if b <= a:
            continue
        for z, w in zip(gx, gw):
            s = a + 0.5 * (b - a) * (1.0 + z)
            val = np.asarray(f(s), dtype=float) * (0.5 * (b - a) * w)
            total = val if total is None else total + val
    return total


def sbar(r, x0, d, n, L):
    """Orbit-averaged shape {node: int_0^1 S_g(x(s)) ds}."""
    acc = {}
    cuts = [0.0] + knot_crossings(r, x0, d, n, L) + [1.0]
    gx, gw = np.polynomial.legendre.leggauss(12)
    for a, b in zip(cuts[:-1], cuts[1:]):
        if b <= a:
            continue
        for z, w in zip(gx, gw):
            s = a + 0.5 * (b - a) * (1.0 + z)
            x = [x0[c] + s * d[c] for c in range(3)]
            for g, v in shape_weights(r, x, n, L).items():
                acc[g] = acc.get(g, 0.0) + v * 0.5 * (b - a) * w
    return acc


def orbit_D(r, x0, d, n, L, A0, A1):
    """[D A]_lj = int_0^1 sum_g A_lg(s) d_j S_g(x(s)) ds,
    A_g(s) = (1 - s) A0_g + s A1_g."""
    def f(s):
        x = [x0[c] + s * d[c] for c in range(3)]
        _, g0 = point_values(r, x, n, L, A0, deriv=True)
        _, g1 = point_values(r, x, n, L, A1, deriv=True)
        return (1.0 - s) * g0 + s * g1
    return orbit_integral(f, r, x0, d, n, L)


def orbit_gather(r, x0, d, n, L, F):
    """sum_g F_g Sbar_g = int_0^1 F_h(x(s)) ds."""
    def f(s):
        x = [x0[c] + s * d[c] for c in range(3)]
        return point_values(r, x, n, L, F)
    return orbit_integral(f, r, x0, d, n, L)


# --------------------------------------------------------------------------
# the unsplit comparison rule (Sec. 4.7, Tables 1-2): one n_q-point
# Gauss-Legendre rule over the whole orbit s in [0, 1], each point weighted
# by the true B-spline values (and gradients) at its own position, i.e. the
# stencil of the cell the point lies in
# --------------------------------------------------------------------------
def unsplit_points(nq):
    """numpy's Gauss-Legendre rule mapped to [0, 1]: (s_q, w_q)."""
    z, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (1.0 + z), 0.5 * w


def unsplit_sbar(r, x0, d, n, L, nq):
    """{node: sum_q w_q S_g(x(s_q))}."""
    acc = {}
    for s, w in zip(*unsplit_points(nq)):
        x = [x0[c] + s * d[c] for c in range(3)]
        for g, v in shape_weights(r, x, n, L).items():
            acc[g] = acc.get(g, 0.0) + v * w
    return acc


def unsplit_gather(r, x0, d, n, L, F, nq):
    """sum_q w_q F_h(x(s_q))."""
    out = np.zeros(F.shape[0])
    for s, w in zip(*unsplit_points(nq)):
        out += w * point_values(r, [x0[c] + s * d[c] for c in range(3)], n, L, F)
    return out


def unsplit_D(r, x0, d, n, L, A0, A1, nq):
    """sum_q w_q [(1 - s_q) grad A0_h + s_q grad A1_h](x(s_q))."""
    out = np.zeros((A0.shape[0], 3))
    for s, w in zip(*unsplit_points(nq)):
        x = [x0[c] + s * d[c] for c in range(3)]
        _, g0 = point_values(r, x, n, L, A0, deriv=True)
        _, g1 = point_values(r, x, n, L, A1, deriv=True)
        out += w * ((1.0 - s) * g0 + s * g1)
    return out
