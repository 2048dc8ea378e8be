"""Pins of the oracle with several particle species.

Every particle carries its own charge q_i and mass m_i in the model (Sec. 2);
the paper's runs use one species.  The pins: relabelling the species (or
splitting one species into two identical ones) changes nothing; negating
every charge leaves the particles unchanged and negates every field, exactly;
a neutral electron-ion plasma conserves energy and keeps the constraints at
roundoff; and the ions of a cold electron-ion plasma raise the Langmuir
frequency to sqrt(1 + m_e / m_i) omega_pe (with the shape factor of the
mode and the frequency map of the implicit midpoint rule).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2606_15035_amd import workloads as W


def run(wl, steps, species=None, qs=None, ms=None, **kw):
    cfg = O.make_cfg(**{**wl.cfg_kwargs(), **kw})
    s = O.OracleSim(cfg, wl.np)
    sp = wl.species if species is None else species
    s.init_species(wl.x, wl.v, sp, wl.qs if qs is None else qs, wl.ms if ms is None else ms,
                   wl.n0)
    for _ in range(steps):
        s.step()
    return s


def test_one_species_split_in_two_is_unchanged():
    wl = W.random_plasma((8, 8, 4), (1.0, 1.0, 0.5), 1500, r=2, dt=0.25, vth=0.06,
                         drift=(0.03, -0.02, 0.01), seed=7)
    a = O.OracleSim(O.make_cfg(**wl.cfg_kwargs()), wl.np)
    a.init_particles(wl.x, wl.v, wl.q, wl.m, wl.n0)
    for _ in range(3):
        a.step()
    sp = (np.arange(wl.np) % 2).astype(np.int32)
    b = run(wl, 3, species=sp, qs=[wl.q, wl.q], ms=[wl.m, wl.m])
    sa, sb = a.get_state(), b.get_state()
    for k in ("x", "v", "vprev", "P", "fields"):
        np.testing.assert_array_equal(sa[k], sb[k])


def test_relabelled_species_are_unchanged():
    wl = W.electron_ion((8, 8, 4), (1.0, 1.0, 0.5), 2000, r=1, dt=0.25, vth=0.06,
                        drift=(0.05, 0.0, 0.0), seed=8)
    a = run(wl, 3)
    b = run(wl, 3, species=1 - wl.species, qs=wl.qs[::-1], ms=wl.ms[::-1])
    sa, sb = a.get_state(), b.get_state()
    for k in ("x", "v", "P", "fields"):
        np.testing.assert_array_equal(sa[k], sb[k])
    # and the species really differ: all particles with the electrons' q/m move otherwise
    c = run(wl, 3, qs=[wl.qs[0], wl.qs[0]], ms=[wl.ms[0], wl.ms[0]])
    assert np.abs(c.get_state()["v"] - sa["v"]).max() > 1e-3 * np.abs(sa["v"]).max()


def test_negated_charges_negate_the_fields_exactly():
    wl = W.electron_ion((8, 8, 4), (1.0, 1.0, 0.5), 2000, r=2, dt=0.25, vth=0.06,
                        drift=(0.05, 0.0, 0.0), seed=9)
    a = run(wl, 3)
    b = run(wl, 3, qs=[-q for q in wl.qs])
    sa, sb = a.get_state(), b.get_state()
    np.testing.assert_array_equal(sa["x"], sb["x"])
    np.testing.assert_array_equal(sa["v"], sb["v"])
    np.testing.assert_array_equal(sa["fields"], -sb["fields"])
    assert np.abs(sa["fields"]).max() > 0.0


@pytest.mark.parametrize("r", [1, 2, 3])
def test_electron_ion_energy_and_constraints(r):
    wl = W.electron_ion((8, 8, 4), (1.0, 1.0, 0.5), 1600, r=r, dt=0.3, vth=0.08,
                        drift=(0.04, -0.03, 0.02), seed=10 + r)
    cfg = O.make_cfg(**{**wl.cfg_kwargs(), "tol": 1e-13, "pmax": 40})
    s = O.OracleSim(cfg, wl.np)
    s.init_species(wl.x, wl.v, wl.species, wl.qs, wl.ms, wl.n0)
    E0 = s.energy()["E_total"]
    for _ in range(6):
        s.step()
        e = s.energy()
        assert abs(e["R_total"]) < 2e-14 * E0, e
        assert abs(e["E_total"] - E0) < 1e-13 * E0
        assert e["RA_max"] < 1e-14 and e["pou_max"] < 1e-14
        assert e["gauge_max"] < 1e-13 and e["gauss_max"] < 1e-11
    assert e["W"] > 1e-4 * E0


@pytest.mark.slow
@pytest.mark.parametrize("mass_ratio,r", [(16.0, 1), (4.0, 2)])
def test_ions_raise_the_langmuir_frequency(mass_ratio, r):
    wl = W.plasma_oscillation(mass_ratio, r=r)
    s = O.OracleSim(O.make_cfg(**wl.cfg_kwargs()), wl.np)
    s.init_species(wl.x, wl.v, wl.species, wl.qs, wl.ms, wl.n0)
    z = []
    for _ in range(wl.steps):
        s.step()
        f = s.get_state()["fields"]
        ph = np.fft.fft(f[0].mean(axis=(1, 2)))
        uh = np.fft.fft(f[5].mean(axis=(1, 2)))
        z.append((1j * W.K1 * ph[1] + uh[1]).imag)  # E_x of mode k1 (sine phase)
    z = np.array(z)
    t = wl.dt * np.arange(1, wl.steps + 1)
    zc = [t[i] - z[i] * (t[i + 1] - t[i]) / (z[i + 1] - z[i])
          for i in range(len(z) - 1) if z[i] * z[i + 1] < 0]
    assert len(zc) >= 6
    omega = math.pi / np.mean(np.diff(zc))
    H = wl.L[0] / wl.n[0]
    sinc = math.sin(W.K1 * H / 2) / (W.K1 * H / 2)
    w_cont = math.sqrt((1.0 + 1.0 / mass_ratio) * sinc ** (2 * (r + 1)))
    w_disc = 2.0 / wl.dt * math.atan(w_cont * wl.dt / 2.0)  # implicit midpoint rule
    assert abs(omega / w_disc - 1.0) < 5e-4, (omega, w_disc)
    # without the ions' response the frequency would be 3% (M = 16) or 12% (M = 4) lower
    assert abs(omega / (w_disc / math.sqrt(1.0 + 1.0 / mass_ratio)) - 1.0) > 1e-2


def test_bad_species_index_is_rejected():
    wl = W.electron_ion((8, 8, 4), (1.0, 1.0, 0.5), 100, r=1, dt=0.25, vth=0.06)
    s = O.OracleSim(O.make_cfg(**wl.cfg_kwargs()), wl.np)
    sp = wl.species.copy()
    sp[5] = 2
    with pytest.raises(ValueError):
        s.init_species(wl.x, wl.v, sp, wl.qs, wl.ms, wl.n0)
