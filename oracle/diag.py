"""FP64 oracle of the paper's diagnostics (TEST INFRASTRUCTURE ONLY).

The results section reports, besides the cycle-averaged profiles: the time and space
averaged isotropic part f0(U)/n_e of the electron distribution, the density of "fast"
electrons with energy above e0 V0 / 4, and profiles at the instant t f = 0.25 of the
field E, n_e, the mean energy U_e = w_e / n_e, the heating rate -e0 E Gamma_e, the
ionisation rate S, the electron particle flux Gamma_e and energy flux Q_e; and the
electron and ion fluxes at the powered electrode against time.  Readings (the paper
defines the quantities, not how a particle code samples them):

* a sample is the completed state at one time level t_n; a diagnostic window adds up the
  samples it is given (every k steps for time averages, once per period at a fixed phase
  for phase-resolved profiles);
* node quantities use the cloud-in-cell weights and node volumes of the moments (dx,
  dx/2 at the electrodes), the constant weight W, and divide by the number of samples;
* U = m_e |v|^2 / (2 e0) in eV; Q_e = sum e0 U v_x; S = sum n_gas sigma_iz(U) |v| (the
  expected ionisation rate of each electron, electron-impact ionisation tables, atoms at
  rest); the heating rate is -e0 E_i Gamma_e,i formed per sample and then averaged; fast
  means U > V0 / 4 (V0 in volts = e0 V0 / 4 in eV) with the amplitude in use;
* f0/n_e: energy histogram of all sampled electrons in bins of width dU over [0, U_max),
  normalised with the isotropic convention n_e = integral f0(U) sqrt(U) dU, so at a bin
  centre U_k: f0/n_e = count_k / (N dU sqrt(U_k)), N all sampled electrons (those at or
  above U_max included), in eV^-3/2.

Pins (tests/test_oracle_diag.py): a Maxwellian load gives f0/n_e = 2 / sqrt(pi) (kT)^-3/2
e^(-U/kT) and mean energy 3 kT / 2; uniform drift gives Gamma_e = n v_d and Q_e = n U v_d
per node; the ionisation rate of a mono-energetic beam is n n_gas sigma(U) v.
"""
import numpy as np

from . import field, xsec
from .constants import E0, ME

E_IONIZATION = 2


def node_volume(cfg):
    dx = cfg.gap_m / cfg.n_cells
    V = np.full(cfg.n_cells + 1, dx)
    V[0] = V[-1] = 0.5 * dx
    return V


class Window:
    """Diagnostic window of one discharge: sums over the samples given to it."""

    def __init__(self, cfg, n_bins=200, u_max_eV=50.0):
        nn = cfg.n_cells + 1
        self.cfg, self.n_bins, self.u_max = cfg, int(n_bins), float(u_max_eV)
        self.sums = {k: np.zeros(nn) for k in ("n", "U", "fx", "q", "s", "fast", "heat", "E")}
        self.hist = np.zeros(self.n_bins)
        self.n_electrons = 0
        self.n_samples = 0

    def add(self, x, v, E_nodes, V0, n_gas):
        """One sample: electron positions x [m], velocities v [N x 3] [m/s], node field E
        [V/m] at the same time level, amplitude in use V0 [V], gas density [m^-3]."""
        cfg = self.cfg
        dx = cfg.gap_m / cfg.n_cells
        x = np.asarray(x, dtype=np.float64)
        v = np.asarray(v, dtype=np.float64)
        g2 = np.einsum("ij,ij->i", v, v)
        U = 0.5 * ME * g2 / E0
        iz = [p for p in cfg.processes if p.kind == E_IONIZATION]
        nu = np.zeros_like(U)
        for p in iz:
            nu += n_gas * xsec.sigma_lookup(p, U) * np.sqrt(g2)
        dep = lambda wgt: field.deposit(x, wgt, dx, cfg.n_cells)   # noqa: E731
        fx = dep(v[:, 0])
        self.sums["n"] += dep(1.0)
        self.sums["U"] += dep(U)
        self.sums["fx"] += fx
        self.sums["q"] += dep(E0 * U * v[:, 0])
        self.sums["s"] += dep(nu)
        self.sums["fast"] += dep((U > V0 / 4.0).astype(np.float64))
        self.sums["heat"] += -E0 * np.asarray(E_nodes, dtype=np.float64) * fx
        self.sums["E"] += np.asarray(E_nodes, dtype=np.float64)
        du = self.u_max / self.n_bins
        k = np.floor(U / du).astype(np.int64)
        self.hist += np.bincount(k[k < self.n_bins], minlength=self.n_bins)[:self.n_bins]
        self.n_electrons += len(U)
        self.n_samples += 1

    def read(self, W):
        """Averages over the samples; W is the superparticle weight per m^2."""
        n = max(self.n_samples, 1)
        V = node_volume(self.cfg)
        S = self.sums
        with np.errstate(invalid="ignore", divide="ignore"):
            mean_U = np.where(S["n"] > 0, S["U"] / S["n"], np.nan)
        du = self.u_max / self.n_bins
        uc = (np.arange(self.n_bins) + 0.5) * du
        eedf = self.hist / (max(self.n_electrons, 1) * du * np.sqrt(uc))
        return dict(n_e=W * S["n"] / (V * n), mean_energy_e=mean_U, flux_e=W * S["fx"] / (V * n),
                    energy_flux_e=W * S["q"] / (V * n), ionisation_rate=W * S["s"] / (V * n),
                    n_fast=W * S["fast"] / (V * n), heating=W * S["heat"] / (V * n), E=S["E"] / n,
                    eedf=eedf, u_centres=uc, n_samples=self.n_samples)
