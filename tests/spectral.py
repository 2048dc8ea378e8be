"""numpy.fft-based periodic spectral operators for the tests.

Independent of the oracle's own DFT: the symbol of d/dx_a is i k_a with
k_a = 2 pi m / L_a, set to zero on the Nyquist index of an even axis, and the
Laplacian is -|k|^2 with that same k (Sec. 3.3 of the paper, with the Nyquist
reading stated in the design notes)."""
from __future__ import annotations

import numpy as np


def kvec(n, L):
    ks = []
    for a in range(3):
        m = np.fft.fftfreq(n[a], d=1.0 / n[a])
        k = 2 * np.pi * m / L[a]
        if n[a] % 2 == 0:
            k[n[a] // 2] = 0.0
        shape = [1, 1, 1]
        shape[a] = n[a]
        ks.append(k.reshape(shape))
    return np.broadcast_arrays(*ks)


def grad(f, n, L):
    k = kvec(n, L)
    fh = np.fft.fftn(f)
    return np.stack([np.real(np.fft.ifftn(1j * k[a] * fh)) for a in range(3)])


def div(F, n, L):
    k = kvec(n, L)
    return np.real(np.fft.ifftn(sum(1j * k[a] * np.fft.fftn(F[a]) for a in range(3))))


def curl(F, n, L):
    k = kvec(n, L)
    Fh = [np.fft.fftn(F[a]) for a in range(3)]
    c = [1j * (k[1] * Fh[2] - k[2] * Fh[1]), 1j * (k[2] * Fh[0] - k[0] * Fh[2]),
         1j * (k[0] * Fh[1] - k[1] * Fh[0])]
    return np.stack([np.real(np.fft.ifftn(x)) for x in c])


def null_modes(n, L):
    k = kvec(n, L)
    return (k[0] == 0) & (k[1] == 0) & (k[2] == 0)


def poisson(rho, n, L, sigma1=1.0):
    """phi with -Lap phi = sigma1 rho, zero on the null modes."""
    k = kvec(n, L)
    k2 = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
    rh = np.fft.fftn(rho)
    ph = np.zeros_like(rh)
    nz = k2 > 0
    ph[nz] = sigma1 * rh[nz] / k2[nz]
    return np.real(np.fft.ifftn(ph))


def project_null(f, n, L):
    """f with its Fourier coefficients removed on every mode where k = 0."""
    fh = np.fft.fftn(f)
    fh[null_modes(n, L)] = 0.0
    return np.real(np.fft.ifftn(fh))


def transverse(F, n, L):
    """Divergence-free part of a vector field (null modes kept)."""
    k = kvec(n, L)
    k2 = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
    Fh = [np.fft.fftn(F[a]) for a in range(3)]
    kf = k[0] * Fh[0] + k[1] * Fh[1] + k[2] * Fh[2]
    out = []
    for a in range(3):
        g = Fh[a].copy()
        nz = k2 > 0
        g[nz] -= k[a][nz] * kf[nz] / k2[nz]
        out.append(np.real(np.fft.ifftn(g)))
    return np.stack(out)


def field_energy(phi, A, U, n, L, sigma1=1.0, sigma2=1.0):
    H = [L[a] / n[a] for a in range(3)]
    dV = H[0] * H[1] * H[2]
    E = -grad(phi, n, L) - U
    Bf = curl(A, n, L)
    return dV * (np.sum(E ** 2) / (2 * sigma1) + np.sum(Bf ** 2) / (2 * sigma2))
