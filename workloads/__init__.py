"""Seeded synthetic workloads for the 1D3V PIC/MCC step of Becker et al. (arXiv:1608.04601).

This module is the only code shared by the HIP path and the CPU oracle.  It holds
discharge parameters and analytic model-gas cross-section tables: pure input data,
none of the method's arithmetic (no weights, gas densities, collision bounds, ...).

Paper basis for the parameter set (Sec. 2, Table "tab:discharge"; Sec. 4.2, Table
"tab:numericalparameters"): gap d, pressure p, gas temperature T_gas, RF amplitude
V0 and frequency f, cell count, time step, initial density and energies, particle
count.  The paper's cross-section data (Biagi He, Phelps Ar; Sec. 4.1) are not
available, so the processes of Table "tab:reactions" are given analytic model
cross sections (constant elastic and charge-exchange, linear-rise excitation and
ionisation that plateau at twice the threshold).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import Tuple

import numpy as np

# Process kinds (Table "tab:reactions"); the integer codes are the C ABI's.
E_ELASTIC, E_EXCITATION, E_IONIZATION, I_ISOTROPIC, I_BACKWARD = range(5)
PROCESS_KINDS = ("e_elastic", "e_excitation", "e_ionization", "i_isotropic", "i_backward")
PROCESS_SPECIES = (0, 0, 0, 1, 1)
# Energy frame of a table (Sec. 4.1: He ion data in centre-of-mass energy, Ar in lab energy).
FRAME_LAB, FRAME_CM = 0, 1

ELECTRON, ION = 0, 1

AMU_AR = 39.948
AMU_HE = 4.002602


@dataclass(frozen=True)
class Process:
    """One collision process: sigma_m2[k] is the cross section at energy k*de_eV."""
    kind: int
    frame: int
    threshold_eV: float
    de_eV: float
    emin_eV: float
    sigma_m2: np.ndarray

    @property
    def species(self) -> int:
        return PROCESS_SPECIES[self.kind]


@dataclass(frozen=True)
class Discharge:
    """One discharge: the problem statement plus the numerical parameters.

    n_super is the initial superparticle count per species (electrons, ions);
    capacity bounds the per-species particle storage; te/ti_init_eV are k_B*T of
    the initial Maxwellians in eV.
    """
    name: str
    gap_m: float
    pressure_Pa: float
    gas_temperature_K: float
    gas_mass_amu: float
    rf_voltage_V: float
    rf_frequency_Hz: float
    dt_s: float
    n_cells: int
    n_init_m3: float
    te_init_eV: float
    ti_init_eV: float
    n_super: Tuple[int, int]
    capacity: Tuple[int, int]
    seed: int
    processes: Tuple[Process, ...]
    sort_every: int = 20
    moments_every: int = 1
    max_births_per_step: int = 65536
    electron_order: int = -1   # periodic electron reordering: 1 by cell, 0 compaction only, -1 automatic
    j0_target_A_m2: float = 0.0   # > 0: V0 is adapted every RF period towards this current amplitude

    @property
    def steps_per_period(self) -> int:
        return max(1, int(round(1.0 / (self.rf_frequency_Hz * self.dt_s))))

    def replace(self, **kw) -> "Discharge":
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------------------
# Analytic model cross sections
# ---------------------------------------------------------------------------

def constant_table(sigma: float, emax_eV: float, de_eV: float) -> np.ndarray:
    n = int(round(emax_eV / de_eV)) + 1
    return np.full(n, float(sigma), dtype=np.float64)


def ramp_table(threshold_eV: float, sigma_max: float, emax_eV: float, de_eV: float) -> np.ndarray:
    """Zero below threshold, linear rise to sigma_max at twice the threshold, then flat."""
    n = int(round(emax_eV / de_eV)) + 1
    eps = np.arange(n, dtype=np.float64) * de_eV
    frac = np.clip((eps - threshold_eV) / threshold_eV, 0.0, 1.0)
    return sigma_max * frac


def argon_like(emax_e_eV: float = 200.0, emax_i_eV: float = 200.0, de_eV: float = 0.1,
               excitation_sigma: float = 1e-20) -> Tuple[Process, ...]:
    """Argon-like model gas: e elastic 1e-19, excitation 11.5 eV, ionisation 15.8 eV rising
    to 3e-20, ion backward (charge exchange) 5e-19, ion tables in lab energy with a 0.1 eV
    floor (Sec. 4.1)."""
    return (
        Process(E_ELASTIC, FRAME_LAB, 0.0, de_eV, 0.0, constant_table(1e-19, emax_e_eV, de_eV)),
        Process(E_EXCITATION, FRAME_LAB, 11.5, de_eV, 0.0,
                ramp_table(11.5, excitation_sigma, emax_e_eV, de_eV)),
        Process(E_IONIZATION, FRAME_LAB, 15.8, de_eV, 0.0, ramp_table(15.8, 3e-20, emax_e_eV, de_eV)),
        Process(I_BACKWARD, FRAME_LAB, 0.0, de_eV, 0.1, constant_table(5e-19, emax_i_eV, de_eV)),
    )


def helium_like(emax_e_eV: float = 400.0, emax_i_eV: float = 400.0, de_eV: float = 0.1) -> Tuple[Process, ...]:
    """Helium-like model gas: e elastic 6e-20, excitation 19.8 eV (1e-21), ionisation
    24.6 eV (3e-21), ion backward 5e-19; ion tables in centre-of-mass energy (Sec. 4.1)."""
    return (
        Process(E_ELASTIC, FRAME_LAB, 0.0, de_eV, 0.0, constant_table(6e-20, emax_e_eV, de_eV)),
        Process(E_EXCITATION, FRAME_LAB, 19.8, de_eV, 0.0, ramp_table(19.8, 1e-21, emax_e_eV, de_eV)),
        Process(E_IONIZATION, FRAME_LAB, 24.6, de_eV, 0.0, ramp_table(24.6, 3e-21, emax_e_eV, de_eV)),
        Process(I_BACKWARD, FRAME_CM, 0.0, de_eV, 0.0, constant_table(5e-19, emax_i_eV, de_eV)),
    )


def _table_top(v0: float) -> float:
    """Table range: twice the RF amplitude, at least 100 eV (no particle gains more)."""
    return float(max(100.0, 2.0 * v0))


F_RF = 13.56e6


def small_argon(seed: int = 0, n_super: int = 20_000) -> Discharge:
    """Plain FP64-checkable discharge: argon-like, 2 cm, 128 cells, 100 V, 20 Pa, 300 K,
    2e4 particles per species, n_init 1e15 m^-3, 2 eV / 0.026 eV, dt = T_rf/400."""
    top = _table_top(100.0)
    return Discharge(
        name="argon_2cm_128c_20Pa_100V", gap_m=0.02, pressure_Pa=20.0, gas_temperature_K=300.0,
        gas_mass_amu=AMU_AR, rf_voltage_V=100.0, rf_frequency_Hz=F_RF, dt_s=1.0 / (F_RF * 400),
        n_cells=128, n_init_m3=1e15, te_init_eV=2.0, ti_init_eV=0.026,
        n_super=(n_super, n_super), capacity=(4 * n_super, 4 * n_super), seed=seed,
        processes=argon_like(top, top), sort_every=20, moments_every=1)


def small_helium(seed: int = 0, n_super: int = 20_000) -> Discharge:
    """Plain FP64-checkable helium discharge (the second statistical parity case):
    helium-like, 2.5 cm, 128 cells, 200 V, 40 Pa, 300 K, 2e4 particles per species,
    n_init 1e15 m^-3, 2 eV / 0.026 eV, dt = T_rf/800 (ion table in the centre-of-mass
    frame, backward ion scattering)."""
    top = _table_top(200.0)
    return Discharge(
        name="helium_2.5cm_128c_40Pa_200V", gap_m=0.025, pressure_Pa=40.0, gas_temperature_K=300.0,
        gas_mass_amu=AMU_HE, rf_voltage_V=200.0, rf_frequency_Hz=F_RF, dt_s=1.0 / (F_RF * 800),
        n_cells=128, n_init_m3=1e15, te_init_eV=2.0, ti_init_eV=0.026,
        n_super=(n_super, n_super), capacity=(4 * n_super, 4 * n_super), seed=seed,
        processes=helium_like(top, top), sort_every=20, moments_every=1)


def production_helium(seed: int = 0, n_super: int = 1_000_000) -> Discharge:
    """Single discharge at production size: helium-like, 2.5 cm, 512 cells, 200 V, 40 Pa,
    1e6 particles per species, dt = T_rf/2000."""
    top = _table_top(200.0)
    return Discharge(
        name="helium_2.5cm_512c_40Pa_200V", gap_m=0.025, pressure_Pa=40.0, gas_temperature_K=300.0,
        gas_mass_amu=AMU_HE, rf_voltage_V=200.0, rf_frequency_Hz=F_RF, dt_s=1.0 / (F_RF * 2000),
        n_cells=512, n_init_m3=1e15, te_init_eV=2.0, ti_init_eV=0.026,
        n_super=(n_super, n_super), capacity=(2 * n_super, 2 * n_super), seed=seed,
        processes=helium_like(top, top), sort_every=20, moments_every=1)


def large_argon(seed: int = 0, n_super: int = 25_000_000) -> Discharge:
    """Large single discharge: argon-like, 80 Pa, 300 V, 3 cm, 4096 cells, 2.5e7 particles
    per species, dt = T_rf/4000.  Reordered every 50 steps (any 50 consecutive steps hold
    exactly one reordering; the reordering does not change results).  Measured wall time per
    step against the interval: 0.456 ms at 10, 0.432 at 20, 0.427 at 25, 0.416 at 50, 0.413 at
    100: past 50 the pass gains less from cell order than the reordering costs."""
    top = _table_top(300.0)
    return Discharge(
        name="argon_3cm_4096c_80Pa_300V", gap_m=0.03, pressure_Pa=80.0, gas_temperature_K=300.0,
        gas_mass_amu=AMU_AR, rf_voltage_V=300.0, rf_frequency_Hz=F_RF, dt_s=1.0 / (F_RF * 4000),
        n_cells=4096, n_init_m3=1e15, te_init_eV=2.0, ti_init_eV=0.026,
        n_super=(n_super, n_super), capacity=(2 * n_super, 2 * n_super), seed=seed,
        processes=argon_like(top, top), sort_every=50, moments_every=1)


def large_argon_periodic(seed: int = 0, n_periodic: int = 25_000_000) -> Discharge:
    """The large argon discharge with the weight of its periodic state: that state's
    cycle-averaged density is about 9.5e15 m^-3 (the stored steady states nearest 80 Pa,
    300 V, 3 cm), so W = 9.5e15 d / n_periodic and the uniform start at 1e15 m^-3 holds
    n_periodic / 9.5 particles per species; storage for 1.6 n_periodic."""
    n0 = int(round(n_periodic * 1e15 / 9.5e15))
    cap = int(1.6 * n_periodic)
    return large_argon(seed=seed, n_super=n0).replace(name="argon_3cm_4096c_80Pa_300V_periodic_weight",
                                                      capacity=(cap, cap), max_births_per_step=1 << 18)


def sweep_argon(n_discharges: int = 64, seed: int = 0) -> Tuple[Discharge, ...]:
    """Pressure/voltage sweep of argon-like discharges drawn from default_rng(seed):
    p ~ U(10, 80) Pa, V0 ~ U(100, 400) V, d ~ U(2, 3) cm, cells ~ U{256..1024} rounded to
    a multiple of 64, particles per species log-uniform in [1e5, 2e6], dt = T_rf/2000.  The
    uniform start ionises strongly in its first periods: storage is 8x the initial count."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_discharges):
        p = float(rng.uniform(10.0, 80.0))
        v0 = float(rng.uniform(100.0, 400.0))
        d = float(rng.uniform(0.02, 0.03))
        nc = int(rng.integers(256, 1025))
        nc = int(max(256, min(1024, 64 * round(nc / 64))))
        npart = int(round(10 ** rng.uniform(5.0, np.log10(2e6))))
        top = _table_top(v0)
        out.append(Discharge(
            name=f"sweep{k:02d}", gap_m=d, pressure_Pa=p, gas_temperature_K=300.0,
            gas_mass_amu=AMU_AR, rf_voltage_V=v0, rf_frequency_Hz=F_RF, dt_s=1.0 / (F_RF * 2000),
            n_cells=nc, n_init_m3=1e15, te_init_eV=2.0, ti_init_eV=0.026,
            n_super=(npart, npart), capacity=(8 * npart, 8 * npart), seed=seed * 1000 + k,
            processes=argon_like(top, top), sort_every=20, moments_every=1, max_births_per_step=1 << 18))
    return tuple(out)


GAS_IDS = ("argon", "helium")


def surrogate_params(n: int, seed: int) -> np.ndarray:
    """Discharge parameters of the surrogate's training (seed 1) and held-out (seed 2)
    draws from default_rng(seed): rows (p [Pa], V0 [V], d [m], gas id 0 argon / 1 helium),
    p ~ U(10, 80), V0 ~ U(100, 400), d ~ U(0.02, 0.03), gas id ~ U{0, 1}."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(10.0, 80.0, n)
    v0 = rng.uniform(100.0, 400.0, n)
    d = rng.uniform(0.02, 0.03, n)
    gas = rng.integers(0, 2, n).astype(np.float64)
    return np.stack([p, v0, d, gas], axis=1)


def surrogate_discharge(params, k: int = 0, seed: int = 0, n_super: int = 20_000, n_cells: int = 128,
                        steps_per_period: int = 1000, capacity_factor: int = 40) -> Discharge:
    """A discharge of the surrogate's family at reduced fidelity: 128 cells, dt = T_rf/1000,
    2e4 particles per species at n_init = 1e15 m^-3 (this fixes the weight), uniform
    Maxwellian start at 2 eV / 0.026 eV; storage for capacity_factor x the initial count,
    since the periodic state's density can be many times n_init."""
    p, v0, d, gas = (float(v) for v in params)
    top = _table_top(v0)
    helium = int(round(gas)) == 1
    return Discharge(
        name=f"{GAS_IDS[int(helium)]}_{p:.1f}Pa_{v0:.0f}V_{100 * d:.2f}cm_{k}", gap_m=d, pressure_Pa=p,
        gas_temperature_K=300.0, gas_mass_amu=AMU_HE if helium else AMU_AR, rf_voltage_V=v0, rf_frequency_Hz=F_RF,
        dt_s=1.0 / (F_RF * steps_per_period), n_cells=n_cells, n_init_m3=1e15, te_init_eV=2.0, ti_init_eV=0.026,
        n_super=(n_super, n_super), capacity=(capacity_factor * n_super, capacity_factor * n_super),
        seed=seed * 100_000 + k, processes=helium_like(top, top) if helium else argon_like(top, top),
        sort_every=20, moments_every=1, max_births_per_step=1 << 18)
