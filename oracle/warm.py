"""Warm-start load from cycle-averaged profiles (TEST INFRASTRUCTURE ONLY).

The paper's periodic state does not depend on the initial density and energy (Sec. 3, on
initial values), so a discharge may start from any state; a warm start loads one that
resembles the periodic state.  Readings (the paper gives no such loader):

* profiles are given on P >= 2 equally spaced points spanning [0, d], including both
  electrodes, and are linear between the points;
* species s gets N_s = round(integral of n_s dx / W) particles of the discharge's
  constant weight W (Sec. 2.5), at positions drawn from the density by inverting its
  cumulative integral (exact for the piecewise-linear density);
* electrons are Maxwellian with k_B T_e = (2/3) <eps_e>(x), ions Maxwellian at the gas
  temperature with mean v_x = Gamma_i(x) / n_i(x) (zero where n_i = 0), all three
  quantities linear between the points;
* random numbers: Philox counters (k, 0, 0 or 1, (s << 8) | 0xFE) for particle k of
  species s (stream 0xFE), ids 0 .. N_s - 1.

Pins (tests/test_oracle_warm.py): a constant profile gives x = d u exactly (u the
position draw); the loaded positions follow the profile's cumulative distribution
(Kolmogorov-Smirnov bound); the velocity moments reproduce T_e, T_gas and the drift.
"""
import numpy as np

from .constants import AMU, E0, KB, ME
from .philox import draw, normal_pair, uniform
from .pic import derive

STREAM_WARM = 0xFE


def cumulative(dens, h):
    """Cumulative integral of the piecewise-linear density at the points (trapezoids)."""
    dens = np.asarray(dens, dtype=np.float64)
    return np.concatenate([[0.0], np.cumsum(0.5 * (dens[:-1] + dens[1:]) * h)])


def count(cfg, dens):
    h = cfg.gap_m / (len(dens) - 1)
    return int(np.floor(cumulative(dens, h)[-1] / derive(cfg).W + 0.5))


def invert(dens, h, c):
    """Position whose cumulative integral is c: segment by search, then the root in [0, 1]
    of a t + (b - a) t^2 / 2 = (c - C_j) / h (a, b the densities at the segment's ends)."""
    dens = np.asarray(dens, dtype=np.float64)
    C = cumulative(dens, h)
    j = np.clip(np.searchsorted(C, c, side="right") - 1, 0, len(dens) - 2)
    a, b = dens[j], dens[j + 1]
    q = (c - C[j]) / h
    disc = np.sqrt(np.maximum(a * a + 2.0 * (b - a) * q, 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(a + disc > 0.0, 2.0 * q / (a + disc), 0.5)
    t = np.clip(t, 0.0, 1.0)
    return j, t


def load_species(cfg, prof, s):
    """(x [m], v [N x 3], ids) of species s (0 electrons, 1 ions)."""
    dens = np.asarray(prof["n_e"] if s == 0 else prof["n_i"], dtype=np.float64)
    P = len(dens)
    h = cfg.gap_m / (P - 1)
    C = cumulative(dens, h)
    n = count(cfg, dens)
    k = np.arange(n, dtype=np.uint64)
    a0, a1, a2, _ = draw(k, 0, s, STREAM_WARM, cfg.seed)
    b0, b1, _, _ = draw(k, 1, s, STREAM_WARM, cfg.seed)
    j, t = invert(dens, h, uniform(a0) * C[-1])
    x = (j + t) * h
    z0, z1 = normal_pair(a1, a2)
    z2, _ = normal_pair(b0, b1)
    if s == 0:
        kT = (2.0 / 3.0) * np.asarray(prof["mean_energy_e"], dtype=np.float64)   # eV
        v2 = E0 * ((1.0 - t) * kT[j] + t * kT[j + 1]) / ME
        u = np.zeros(n)
    else:
        M = cfg.gas_mass_amu * AMU
        v2 = np.full(n, KB * cfg.gas_temperature_K / M)
        ni = np.asarray(prof["n_i"], dtype=np.float64)
        flux = np.asarray(prof["flux_i"], dtype=np.float64)
        drift = np.divide(flux, ni, out=np.zeros(P), where=ni > 0.0)
        u = (1.0 - t) * drift[j] + t * drift[j + 1]
    vth = np.sqrt(v2)
    v = np.stack([vth * z0 + u, vth * z1, vth * z2], axis=1)
    return x, v, k
