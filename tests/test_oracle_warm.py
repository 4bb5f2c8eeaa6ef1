"""Pins of the oracle's warm-start loader against what the definitions fix: the constant
profile's exact positions, the distribution of the positions (Kolmogorov-Smirnov), and
the velocity moments (temperatures and drift)."""
import numpy as np

import workloads as W
from oracle import warm
from oracle.constants import AMU, E0, KB, ME
from oracle.philox import draw, uniform
from oracle.pic import derive


def _disc(n=40_000):
    return W.small_argon(seed=21, n_super=n)


def _profiles(P=129, d=0.02):
    z = np.linspace(0.0, d, P)
    ne = 1e15 * np.sin(np.pi * z / d) ** 2
    ni = 1e15 * (0.2 + np.sin(np.pi * z / d))
    eps = 2.0 + 6.0 * (z / d)
    flux = 1e19 * (2.0 * z / d - 1.0)
    return dict(n_e=ne, n_i=ni, mean_energy_e=eps, flux_i=flux), z


def test_constant_profile_gives_uniform_positions_exactly():
    disc = _disc()
    P = 17
    prof = dict(n_e=np.full(P, disc.n_init_m3), n_i=np.full(P, disc.n_init_m3),
                mean_energy_e=np.full(P, 3.0), flux_i=np.zeros(P))
    for s in (0, 1):
        x, v, k = warm.load_species(disc, prof, s)
        assert len(x) == disc.n_super[s]     # n_init d / W particles
        a0 = draw(k, 0, s, warm.STREAM_WARM, disc.seed)[0]
        np.testing.assert_allclose(x, disc.gap_m * uniform(a0), rtol=1e-12, atol=1e-18)


def test_positions_follow_the_profile():
    disc = _disc()
    prof, z = _profiles(d=disc.gap_m)
    for s, key in ((0, "n_e"), (1, "n_i")):
        x, _, _ = warm.load_species(disc, prof, s)
        n = len(x)
        C = warm.cumulative(prof[key], z[1] - z[0])
        expect = np.sum(prof[key][:-1] + prof[key][1:]) * 0.5 * (z[1] - z[0]) / derive(disc).W
        assert abs(n - expect) <= 1.0
        # empirical CDF against the exact piecewise-quadratic CDF at many points
        q = np.linspace(0.0, disc.gap_m, 1001)[1:-1]
        j = np.minimum((q / (z[1] - z[0])).astype(int), len(z) - 2)
        t = q / (z[1] - z[0]) - j
        a, b = prof[key][j], prof[key][j + 1]
        F = (C[j] + (z[1] - z[0]) * (a * t + 0.5 * (b - a) * t * t)) / C[-1]
        emp = np.searchsorted(np.sort(x), q) / n
        assert np.max(np.abs(emp - F)) <= 1.63 / np.sqrt(n)    # KS, 1 % level


def test_velocity_moments():
    disc = _disc(100_000)
    P = 9
    prof = dict(n_e=np.full(P, 1e15), n_i=np.full(P, 1e15), mean_energy_e=np.full(P, 4.5),
                flux_i=np.full(P, 1e15 * 300.0))
    _, ve, _ = warm.load_species(disc, prof, 0)
    _, vi, _ = warm.load_species(disc, prof, 1)
    n = len(ve)
    # k T_e = (2/3) 4.5 eV = 3 eV per component; ions at the gas temperature, drifting 300 m/s
    var_e = E0 * 3.0 / ME
    assert np.all(np.abs(ve.var(axis=0) / var_e - 1.0) <= 5 * np.sqrt(2.0 / n))
    var_i = KB * disc.gas_temperature_K / (disc.gas_mass_amu * AMU)
    assert np.all(np.abs(vi.var(axis=0) / var_i - 1.0) <= 5 * np.sqrt(2.0 / n))
    assert abs(vi[:, 0].mean() - 300.0) <= 5 * np.sqrt(var_i / n)
    assert np.all(np.abs(vi[:, 1:].mean(axis=0)) <= 5 * np.sqrt(var_i / n))
