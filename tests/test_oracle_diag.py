"""Pins of the oracle's diagnostics against closed forms: a Maxwellian's f0/n_e and mean
energy, the fluxes and heating of a uniformly drifting population, and the ionisation
rate and fast-electron density of a mono-energetic beam on the model gas's plateau."""
import numpy as np

import workloads as W
from oracle import diag
from oracle.constants import E0, KB, ME
from oracle.pic import derive


def _disc():
    return W.small_argon(seed=3, n_super=1000)


def _uniform_x(rng, n, d):
    return rng.uniform(0.0, d, n)


def test_maxwellian_eedf_and_mean_energy():
    disc = _disc()
    rng = np.random.default_rng(0)
    kT, n = 3.0, 400_000
    x = _uniform_x(rng, n, disc.gap_m)
    v = rng.normal(0.0, np.sqrt(kT * E0 / ME), (n, 3))
    win = diag.Window(disc, n_bins=120, u_max_eV=30.0)
    win.add(x, v, np.zeros(disc.n_cells + 1), disc.rf_voltage_V, 1.0)
    r = win.read(derive(disc).W)
    u = r["u_centres"]
    expect = 2.0 / np.sqrt(np.pi) * kT ** -1.5 * np.exp(-u / kT)
    counts = win.hist
    ok = counts > 2000
    rel = np.abs(r["eedf"][ok] / expect[ok] - 1.0)
    assert np.all(rel <= 5.0 / np.sqrt(counts[ok]) + 0.01)
    # normalisation: integral f0/n_e sqrt(U) dU is the fraction sampled below U_max
    frac = np.sum(r["eedf"] * np.sqrt(u) * (u[1] - u[0]))
    assert abs(frac - np.mean(0.5 * ME * np.sum(v * v, axis=1) / E0 < 30.0)) <= 1e-12
    inner = slice(2, -2)
    assert np.all(np.abs(r["mean_energy_e"][inner] / (1.5 * kT) - 1.0) <= 0.03)
    dens = derive(disc).W * n / disc.gap_m
    assert np.all(np.abs(r["n_e"][inner] / dens - 1.0) <= 0.05)


def test_drift_fluxes_and_heating_are_exact():
    disc = _disc()
    rng = np.random.default_rng(1)
    n, vd, Ec = 50_000, 2.0e5, -300.0
    x = _uniform_x(rng, n, disc.gap_m)
    v = np.zeros((n, 3))
    v[:, 0] = vd
    win = diag.Window(disc)
    E = np.full(disc.n_cells + 1, Ec)
    win.add(x, v, E, disc.rf_voltage_V, 1.0)
    win.add(x, v, E, disc.rf_voltage_V, 1.0)
    r = win.read(derive(disc).W)
    U = 0.5 * ME * vd * vd / E0
    np.testing.assert_allclose(r["flux_e"], r["n_e"] * vd, rtol=1e-12)
    np.testing.assert_allclose(r["energy_flux_e"], r["n_e"] * E0 * U * vd, rtol=1e-12)
    np.testing.assert_allclose(r["heating"], -E0 * Ec * r["n_e"] * vd, rtol=1e-12)
    np.testing.assert_allclose(r["E"], Ec, rtol=1e-15)
    assert r["n_samples"] == 2


def test_beam_ionisation_rate_and_fast_electrons():
    disc = _disc()
    rng = np.random.default_rng(2)
    n, U0 = 30_000, 50.0      # on the argon-like ionisation plateau, 3e-20 m^2
    v0 = np.sqrt(2.0 * U0 * E0 / ME)
    x = _uniform_x(rng, n, disc.gap_m)
    dirs = rng.normal(size=(n, 3))
    v = v0 * dirs / np.linalg.norm(dirs, axis=1)[:, None]
    ng = disc.pressure_Pa / (KB * disc.gas_temperature_K)
    for V0, all_fast in ((100.0, True), (250.0, False)):   # fast above V0 / 4 = 25 or 62.5 eV
        win = diag.Window(disc)
        win.add(x, v, np.zeros(disc.n_cells + 1), V0, ng)
        r = win.read(derive(disc).W)
        np.testing.assert_allclose(r["ionisation_rate"], r["n_e"] * ng * 3e-20 * v0, rtol=1e-9)
        np.testing.assert_allclose(r["n_fast"], r["n_e"] if all_fast else 0.0, rtol=1e-12, atol=0)
