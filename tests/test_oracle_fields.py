"""Pins of the oracle's mesh arithmetic (no GPU): DFT and symbols against
numpy.fft, the CN vacuum wave against its closed form, Theorem 1 (gauge and
Gauss preservation for any current), and the CN field-energy balance
(eq. field-energy-final)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2606_15035_amd import workloads as W
from tests import spectral as SP

N = (8, 6, 4)
L = (1.3, 0.9, 0.7)


def sim(dt=0.1, n=N, Lb=L, kappa=1.0, sigma2=1.0):
    return O.OracleSim(O.make_cfg(n=n, L=Lb, dt=dt, r=1, kappa=kappa, sigma1=kappa ** 2 * sigma2,
                                  sigma2=sigma2), 0)


def test_dft_matches_numpy_fft():
    S = sim()
    rng = np.random.default_rng(1)
    f = rng.normal(size=N) + 1j * rng.normal(size=N)
    np.testing.assert_allclose(S.dft3(f, -1), np.fft.fftn(f), atol=1e-12)
    np.testing.assert_allclose(S.dft3(f, +1), np.fft.ifftn(f), atol=1e-14)


def test_ktilde_symbols():
    S = sim()
    k = S.ktilde()
    ref = SP.kvec(N, L)
    for a in range(3):
        np.testing.assert_allclose(k[a], ref[a], atol=1e-13)


def test_config_validation():
    bad = O.make_cfg(n=N, L=L, dt=0.1, kappa=2.0, sigma1=1.0, sigma2=1.0)  # sigma1 != kappa^2 sigma2
    assert O.lib().orc_check_config(bad) != 0
    assert O.lib().orc_check_config(O.make_cfg(n=N, L=L, dt=0.1, r=4)) != 0
    assert O.lib().orc_check_config(O.make_cfg(n=N, L=L, dt=0.1, r=3)) == 0
    assert O.lib().orc_check_config(O.make_cfg(n=N, L=L, dt=0.1, kappa=2.0, sigma1=4.0, sigma2=1.0)) == 0


@pytest.mark.parametrize("kappa", [1.0, 2.5])
def test_cn_vacuum_wave_closed_form(kappa):
    """Source-free CN of one transverse mode is a rotation by theta with
    tan(theta/2) = kappa |k| dt / 2: A_n = cos(n theta), U_n = -w sin(n theta)."""
    dt = 0.3
    S = sim(dt=dt, kappa=kappa)
    nc = int(np.prod(N))
    x = np.arange(N[0]) * L[0] / N[0]
    k = 2 * math.pi / L[0]
    fields = np.zeros((9,) + N)
    fields[3] = np.cos(k * x).reshape(-1, 1, 1)  # A_y(x): transverse, gauge-free
    S.set_state(None, None, None, None, fields, q=-1.0, m=1.0)
    w = kappa * k
    theta = 2 * math.atan(w * dt / 2)
    Jz = np.zeros((3,) + N)
    for nstep in range(1, 25):
        S.field_solve(Jz)
        f = S.get_state()["fields"]
        np.testing.assert_allclose(f[3][:, 0, 0], math.cos(nstep * theta) * np.cos(k * x), atol=1e-13)
        np.testing.assert_allclose(f[6][:, 0, 0], -w * math.sin(nstep * theta) * np.cos(k * x),
                                   atol=1e-12 * w)
    assert nc > 0


def consistent_state(seed, n=N, Lb=L, sigma1=1.0):
    """phi from Poisson of a neutral rho (zero on the k = 0 modes), psi = 0,
    transverse random A and U: satisfies the Lorenz gauge and Gauss's law."""
    rho = SP.project_null(W.random_fields(n, 1, seed=seed)[0], n, Lb)
    phi = SP.poisson(rho, n, Lb, sigma1)
    A = SP.transverse(W.random_fields(n, 3, seed=seed + 1), n, Lb)
    U = SP.transverse(W.random_fields(n, 3, seed=seed + 2), n, Lb)
    f = np.zeros((9,) + n)
    f[0] = phi
    f[2:5] = A
    f[5:8] = U
    f[8] = rho
    return f


@pytest.mark.parametrize("kappa", [1.0, 2.5])
def test_theorem1_gauge_and_gauss_preserved_for_any_current(kappa):
    S = sim(dt=0.2, kappa=kappa)
    S.set_state(None, None, None, None, consistent_state(5, sigma1=kappa ** 2), q=-1.0, m=1.0)
    e = S.energy()
    assert e["gauge_max"] < 1e-13 and e["gauss_max"] < 1e-12
    for it in range(10):
        J = 3.0 * W.random_fields(N, 3, seed=100 + it)  # arbitrary, with longitudinal parts
        S.field_solve(J)
        e = S.energy()
        f = S.get_state()["fields"]
        assert np.abs(f).max() > 0.1
        assert e["gauge_max"] < 2e-13, e
        assert e["gauss_max"] < 2e-12, e
    # the residuals are what the definitions say
    G = f[1] / kappa ** 2 + SP.div(f[2:5], N, L)
    R = SP.div(-SP.grad(f[0], N, L) - f[5:8], N, L) - kappa ** 2 * f[8]
    assert abs(np.abs(G).max() - e["gauge_max"]) < 1e-12
    assert abs(np.abs(R).max() - e["gauss_max"]) < 1e-11


def test_gauss_broken_by_inconsistent_charge():
    """Negative control: advancing rho without the continuity equation (here:
    a state whose rho disagrees with phi) shows up in R_h."""
    S = sim()
    f = consistent_state(7)
    f[8] += 0.1 * SP.project_null(W.random_fields(N, 1, seed=99)[0], N, L)
    S.set_state(None, None, None, None, f, q=-1.0, m=1.0)
    assert S.energy()["gauss_max"] > 1e-3


@pytest.mark.parametrize("kappa,sigma2", [(1.0, 1.0), (2.0, 0.7)])
def test_cn_field_energy_balance(kappa, sigma2):
    """W^{n+1} - W^n = -dt sum_g J . E^{n+1/2} dV for a gauge-consistent state."""
    dt = 0.15
    S = sim(dt=dt, kappa=kappa, sigma2=sigma2)
    S.set_state(None, None, None, None, consistent_state(11, sigma1=kappa ** 2 * sigma2), q=-1.0,
                m=1.0)
    dV = np.prod([L[a] / N[a] for a in range(3)])
    for it in range(6):
        f0 = S.get_state()["fields"]
        W0 = S.energy()["W"]
        np.testing.assert_allclose(W0, SP.field_energy(f0[0], f0[2:5], f0[5:8], N, L,
                                                       kappa ** 2 * sigma2, sigma2), rtol=1e-13)
        J = 20.0 * W.random_fields(N, 3, seed=200 + it)
        S.field_solve(J)
        f1 = S.get_state()["fields"]
        W1 = S.energy()["W"]
        E0 = -SP.grad(f0[0], N, L) - f0[5:8]
        E1 = -SP.grad(f1[0], N, L) - f1[5:8]
        work = dt * np.sum(J * 0.5 * (E0 + E1)) * dV
        assert abs(W1 - W0 + work) < 1e-13 * max(W0, W1), (W1 - W0, -work)
        # the balance is not trivial: the field energy really changes
        assert abs(W1 - W0) > 1e-4 * W0
