"""The PIC/MCC step, written out in FP64 (Sec. 2.5 "PIC/MCC simulation procedure").

One step n -> n+1 (t_n = n dt), in the paper's order (velocity Verlet, Sec. 2.5):
  1. gather a^n = (q/m) E^n(x^n) by cloud-in-cell;
  2. drift x^{n+1} = x^n + v_x^n dt + a^n dt^2 / 2 (1d3v: only v_x feels the field);
  3. absorb every particle with x <= 0 or x >= d, counted per electrode (Sec. 2.2, 2.5:
     full absorption, no reflection, no secondary emission);
  4. deposit the survivors' charge, solve Poisson with phi_0 = V0 sin(2 pi f t_{n+1}),
     phi_{N_c} = 0, and form E^{n+1} (Sec. 2, 2.2);
  5. complete the kick v_x^{n+1} = v_x^n + (a^n + a^{n+1}) dt / 2;
  6. null-collision MCC on the particles alive now (Sec. 2.5): isotropic scattering
     except backward ion-atom scattering, ionisation energy shared equally;
  7. append the ionisation products, ids in ascending order of the parent id;
  8. sample the moments on the end-of-step state.

Readings where the paper is silent (units SI, energies in eV):
  * one constant superparticle weight W = n_init d / N_e(0) per m^2 for both species
    (Sec. 2.5: constant weight; Sec. 4.2: uniform initial density);
  * n_gas = p / (k_B T_gas) (Sec. 2.1); ion mass = gas mass;
  * the initial state is a uniform quasi-neutral load with Maxwellian velocities whose
    k_B T is the configured value in eV (Sec. 2.2, Sec. 4.2);
  * electron-atom collisions see an atom at rest; ion-atom collisions see an atom drawn
    from the gas Maxwellian; "isotropic" means isotropic in the centre-of-mass frame;
    "backward" means the ion leaves with the atom's velocity;
  * the new electron and ion of an ionisation sit at the parent's position; the new ion
    is drawn from the gas Maxwellian; products are first moved in the next step;
  * J^{n+1/2} = eps0 (E_0^{n+1} - E_0^n)/dt + e0 W (N_e,abs,0 - N_i,abs,0)/dt (Sec. 2.2).
"""
from dataclasses import dataclass

import numpy as np

from . import field, xsec
from .constants import AMU, E0, EPS0, KB, ME
from .philox import (STREAM_COLLISION, STREAM_LOAD, STREAM_NEWION, STREAM_SCATTER, STREAM_TARGET,
                     direction, draw, normal_pair, uniform)

ELECTRON, ION = 0, 1
E_ELASTIC, E_EXCITATION, E_IONIZATION, I_ISOTROPIC, I_BACKWARD = range(5)
_SPECIES_OF_KIND = (0, 0, 0, 1, 1)


@dataclass
class Derived:
    dx: float
    n_gas: float
    W: float
    M: float
    m: tuple
    q: tuple
    v_T: float
    numax: tuple
    T: tuple
    p_null: tuple
    steps_per_period: int


def derive(cfg) -> Derived:
    """Derived constants (Sec. 2.1 gas density; Sec. 2.5 constant weight)."""
    dx = cfg.gap_m / cfg.n_cells
    n_gas = cfg.pressure_Pa / (KB * cfg.gas_temperature_K)
    if cfg.n_super[0] <= 0:
        raise ValueError("the weight needs a positive initial electron count")
    W = cfg.n_init_m3 * cfg.gap_m / cfg.n_super[0]
    M = cfg.gas_mass_amu * AMU
    m = (ME, M)
    q = (-E0, E0)
    v_T = np.sqrt(KB * cfg.gas_temperature_K / M)
    numax, T, pn = [], [], []
    for s in (ELECTRON, ION):
        procs = [p for p in cfg.processes if _SPECIES_OF_KIND[p.kind] == s]
        nm = xsec.nu_max(procs, m[s], M, n_gas)
        t, p = xsec.candidate_threshold(nm, cfg.dt_s)
        numax.append(nm)
        T.append(t)
        pn.append(p)
    spp = max(1, int(round(1.0 / (cfg.rf_frequency_Hz * cfg.dt_s))))
    return Derived(dx, n_gas, W, M, m, q, v_T, tuple(numax), tuple(T), tuple(pn), spp)


class _Species:
    def __init__(self, x, v, ids, next_id):
        self.x = np.asarray(x, dtype=np.float64)
        self.v = np.asarray(v, dtype=np.float64).reshape(-1, 3)
        self.id = np.asarray(ids, dtype=np.uint64)
        self.next_id = int(next_id)

    def keep(self, mask):
        self.x, self.v, self.id = self.x[mask], self.v[mask], self.id[mask]


class Oracle:
    """FP64 PIC/MCC discharge.  ``fixed_field`` (node array) replaces the Poisson field in
    every gather (used to pin the pusher); the charge is still deposited."""

    def __init__(self, cfg, load=True, fixed_field=None):
        self.cfg = cfg
        self.d = derive(cfg)
        self.fixed_field = None if fixed_field is None else np.asarray(fixed_field, dtype=np.float64)
        self.n = 0
        self.sp = [_Species([], [], [], 0), _Species([], [], [], 0)]
        self.procs = list(cfg.processes)
        self.coll = np.zeros(len(self.procs), dtype=np.int64)
        self.violations = np.zeros(2, dtype=np.int64)
        self.absorbed_total = np.zeros((2, 2), dtype=np.int64)
        self.J = 0.0
        # RF amplitude; with a target current amplitude J0 it is adapted once per whole RF
        # period as V0 <- V0 J0 / J_calc, J_calc the period's max |J| (Sec. 2, Eq.
        # "adaptivevoltage"), otherwise it stays the prescribed value
        self.V0 = float(cfg.rf_voltage_V)
        self.last = {}
        if load:
            self._load()
        self._field_at(self.n)
        self.reset_moments()

    # ---------------------------------------------------------------- state
    def _load(self):
        """Uniform quasi-neutral load with Maxwellian velocities (Sec. 2.2 initial values)."""
        cfg, d = self.cfg, self.d
        Te = (cfg.te_init_eV, cfg.ti_init_eV)
        for s in (ELECTRON, ION):
            n = int(cfg.n_super[s])
            k = np.arange(n, dtype=np.uint64)
            a0, a1, a2, _ = draw(k, 0, s, STREAM_LOAD, cfg.seed)
            b0, b1, _, _ = draw(k, 1, s, STREAM_LOAD, cfg.seed)
            x = cfg.gap_m * uniform(a0)
            z0, z1 = normal_pair(a1, a2)
            z2, _ = normal_pair(b0, b1)
            vth = np.sqrt(E0 * Te[s] / d.m[s])
            self.sp[s] = _Species(x, vth * np.stack([z0, z1, z2], axis=1), k, n)

    def set_state(self, step, species):
        """species: two dicts with x, vx, vy, vz, id, next_id.  Recomputes E at t_step."""
        self.n = int(step)
        for s in (ELECTRON, ION):
            p = species[s]
            v = np.stack([np.asarray(p["vx"], np.float64), np.asarray(p["vy"], np.float64),
                          np.asarray(p["vz"], np.float64)], axis=1)
            self.sp[s] = _Species(p["x"], v, p["id"], p["next_id"])
        self._field_at(self.n)

    def state(self, s):
        S = self.sp[s]
        o = np.argsort(S.id, kind="stable")
        return dict(x=S.x[o], vx=S.v[o, 0], vy=S.v[o, 1], vz=S.v[o, 2], id=S.id[o], next_id=S.next_id)

    # ---------------------------------------------------------------- field
    def _charge(self):
        d = self.d
        Q = np.zeros(self.cfg.n_cells + 1)
        for s in (ELECTRON, ION):
            Q += field.deposit(self.sp[s].x, d.q[s] * d.W, d.dx, self.cfg.n_cells)
        return Q

    def _field_at(self, step):
        """Deposit, solve with phi_0 = V0 sin(2 pi f t_step), form E (Sec. 2, 2.2)."""
        cfg, d = self.cfg, self.d
        self.Q = self._charge()
        phi0 = self.V0 * np.sin(2.0 * np.pi * cfg.rf_frequency_Hz * step * cfg.dt_s)
        self.phi = field.solve_poisson(self.Q, d.dx, phi0, 0.0)
        self.E = field.node_field(self.phi, self.Q, d.dx)
        self.sigma0 = EPS0 * self.E[0]
        self.sigmad = -EPS0 * self.E[-1]

    def _gather_E(self, x):
        E = self.E if self.fixed_field is None else self.fixed_field
        return field.gather(E, x, self.d.dx, self.cfg.n_cells)

    # ---------------------------------------------------------------- step
    def step(self):
        cfg, d = self.cfg, self.d
        dt = cfg.dt_s
        n = self.n
        acc = [None, None]
        absorbed = np.zeros((2, 2), dtype=np.int64)
        alive_at_start = sum(len(self.sp[s].x) for s in (ELECTRON, ION))
        for s in (ELECTRON, ION):
            S = self.sp[s]
            a = d.q[s] / d.m[s] * self._gather_E(S.x)
            S.x = S.x + S.v[:, 0] * dt + 0.5 * a * dt * dt
            lo = S.x <= 0.0
            hi = S.x >= cfg.gap_m
            absorbed[s] = (int(lo.sum()), int(hi.sum()))
            keep = ~(lo | hi)
            S.keep(keep)
            acc[s] = a[keep]
        E0_old = self.E[0]
        self._field_at(n + 1)
        self.J = EPS0 * (self.E[0] - E0_old) / dt + E0 * d.W * (absorbed[0, 0] - absorbed[1, 0]) / dt
        for s in (ELECTRON, ION):
            S = self.sp[s]
            a2 = d.q[s] / d.m[s] * self._gather_E(S.x)
            S.v[:, 0] += 0.5 * (acc[s] + a2) * dt
        self.absorbed_total += absorbed
        self.last = {"absorbed": absorbed, "alive_at_start": alive_at_start}
        parents = self._mcc(n + 1)
        self._births(n + 1, parents)
        self.n = n + 1
        self._accumulate(absorbed)

    # ---------------------------------------------------------------- collisions
    def _mcc(self, step_field):
        """Null-collision MCC (Sec. 2.5) with counters (id, 0, step_field, tag).  Returns the
        ionising electrons' (ids, x, v_child_e, v_child_i)."""
        cfg, d = self.cfg, self.d
        ion_products = []
        for s in (ELECTRON, ION):
            S = self.sp[s]
            procs = [(j, p) for j, p in enumerate(self.procs) if _SPECIES_OF_KIND[p.kind] == s]
            w0, w1, _, _ = draw(S.id, step_field, s, STREAM_COLLISION, cfg.seed)
            cand = np.nonzero((w0 >> np.uint64(8)) < np.uint64(d.T[s]))[0]
            ids = S.id[cand]
            v = S.v[cand]
            if s == ION:
                b0, b1, b2, b3 = draw(ids, step_field, s, STREAM_TARGET, cfg.seed)
                z0, z1 = normal_pair(b0, b1)
                z2, _ = normal_pair(b2, b3)
                vt = d.v_T * np.stack([z0, z1, z2], axis=1)
            else:
                vt = np.zeros_like(v)
            g = v - vt
            g2 = np.einsum("ij,ij->i", g, g)
            gm = np.sqrt(g2)
            R = uniform(w1[cand]) * d.numax[s]
            c = np.zeros(len(cand))
            sel = np.full(len(cand), -1, dtype=np.int64)
            margin = np.full(len(cand), np.inf)
            for j, p in procs:
                eps = xsec.energy_factor(p, d.m[s], d.M) * g2
                c = c + d.n_gas * xsec.sigma_lookup(p, eps) * gm
                margin = np.minimum(margin, np.abs(R - c))
                hit = (sel < 0) & (R < c)
                sel[hit] = j
            self.violations[s] += int((c > d.numax[s]).sum())
            rec = dict(candidates=ids.copy(), selected=sel.copy(), margin=margin, nu=c,
                       v_before=v.copy(), v_target=vt)
            hit = np.nonzero(sel >= 0)[0]
            c0, c1, c2, c3 = draw(ids[hit], step_field, s, STREAM_SCATTER, cfg.seed)
            n1 = direction(c0, c1)
            n2 = direction(c2, c3)
            vnew = v.copy()
            kinds = np.array([self.procs[j].kind for j in sel[hit]], dtype=np.int64)
            vh, gh, g2h, vth = v[hit], g[hit], g2[hit], vt[hit]
            gmh = np.sqrt(g2h)
            out = vh.copy()
            mm = d.m[s]
            # elastic, two-body, isotropic in the centre-of-mass frame
            for kind in (E_ELASTIC, I_ISOTROPIC):
                k = kinds == kind
                V = (mm * vh[k] + d.M * vth[k]) / (mm + d.M)
                out[k] = V + (d.M / (mm + d.M)) * gmh[k, None] * n1[k]
            # excitation: the threshold energy is lost, new direction isotropic
            k = kinds == E_EXCITATION
            if k.any():
                thr = np.array([self.procs[j].threshold_eV for j in sel[hit][k]])
                eps = 0.5 * mm * g2h[k] / E0
                out[k] = np.sqrt(2.0 * E0 * np.maximum(eps - thr, 0.0) / mm)[:, None] * n1[k]
            # ionisation: the remaining energy is shared equally by the two electrons
            k = kinds == E_IONIZATION
            if k.any():
                thr = np.array([self.procs[j].threshold_eV for j in sel[hit][k]])
                eps = 0.5 * mm * g2h[k] / E0
                sp = np.sqrt(E0 * np.maximum(eps - thr, 0.0) / mm)
                out[k] = sp[:, None] * n1[k]
                pid = ids[hit][k]
                d0, d1, d2, d3 = draw(pid, step_field, s, STREAM_NEWION, cfg.seed)
                y0, y1 = normal_pair(d0, d1)
                y2, _ = normal_pair(d2, d3)
                ion_products.append((pid, S.x[cand[hit][k]].copy(), sp[:, None] * n2[k],
                                     d.v_T * np.stack([y0, y1, y2], axis=1)))
            # backward ion-atom scattering: the ion takes the atom's velocity
            k = kinds == I_BACKWARD
            out[k] = vth[k]
            vnew[hit] = out
            S.v[cand] = vnew
            for j in sel[hit]:
                self.coll[j] += 1
            rec["v_after"] = vnew
            self.last[f"mcc{s}"] = rec
        if ion_products:
            pid = np.concatenate([p[0] for p in ion_products])
            return (pid, np.concatenate([p[1] for p in ion_products]),
                    np.concatenate([p[2] for p in ion_products]), np.concatenate([p[3] for p in ion_products]))
        return (np.zeros(0, np.uint64), np.zeros(0), np.zeros((0, 3)), np.zeros((0, 3)))

    def _births(self, step_field, products):
        """Append ionisation products; the k-th parent in ascending id order gives ids
        next_id_e + k and next_id_i + k."""
        pid, x, ve, vi = products
        o = np.argsort(pid, kind="stable")
        pid, x, ve, vi = pid[o], x[o], ve[o], vi[o]
        nb = len(pid)
        for s, v in ((ELECTRON, ve), (ION, vi)):
            S = self.sp[s]
            if S.next_id + nb > 2 ** 32:
                raise OverflowError("particle ids exhausted")
            new_ids = np.arange(S.next_id, S.next_id + nb, dtype=np.uint64)
            S.x = np.concatenate([S.x, x])
            S.v = np.concatenate([S.v, v.reshape(-1, 3)])
            S.id = np.concatenate([S.id, new_ids])
            S.next_id += nb
        self.last["births"] = dict(parent=pid, child_e=np.arange(self.sp[0].next_id - nb, self.sp[0].next_id),
                                   child_i=np.arange(self.sp[1].next_id - nb, self.sp[1].next_id))

    # ---------------------------------------------------------------- moments
    def reset_moments(self):
        nn = self.cfg.n_cells + 1
        self.m_dens = np.zeros((2, nn))
        self.m_energy = np.zeros(nn)
        self.m_flux = np.zeros(nn)
        self.m_phi = np.zeros(nn)
        self.n_samples = 0
        self.n_window_steps = 0
        self.absorbed_window = np.zeros((2, 2), dtype=np.int64)
        self.J_max_sum = 0.0
        self.n_periods = 0
        self.J_period_max = 0.0
        self.period_valid = (self.n % self.d.steps_per_period) == 0

    def _accumulate(self, absorbed):
        """Window sums on the end-of-step state (moments every M steps)."""
        cfg, d = self.cfg, self.d
        self.n_window_steps += 1
        self.absorbed_window += absorbed
        self.J_period_max = max(self.J_period_max, abs(self.J))
        if self.n % d.steps_per_period == 0:
            if self.period_valid:
                self.J_max_sum += self.J_period_max
                self.n_periods += 1
                j0 = getattr(cfg, "j0_target_A_m2", 0.0)
                if j0 > 0.0 and self.J_period_max > 0.0:
                    self.V0 *= j0 / self.J_period_max
            self.J_period_max = 0.0
            self.period_valid = True
        if self.n % cfg.moments_every != 0:
            return
        self.n_samples += 1
        nc = cfg.n_cells
        for s in (ELECTRON, ION):
            S = self.sp[s]
            self.m_dens[s] += field.deposit(S.x, 1.0, d.dx, nc)
        Se = self.sp[ELECTRON]
        eps = 0.5 * ME * np.einsum("ij,ij->i", Se.v, Se.v) / E0
        self.m_energy += field.deposit(Se.x, eps, d.dx, nc)
        Si = self.sp[ION]
        self.m_flux += field.deposit(Si.x, Si.v[:, 0], d.dx, nc)
        self.m_phi += self.phi

    def moments(self):
        """Window averages: densities and ion flux per node volume (dx inside, dx/2 at the
        electrodes), mean electron energy as a ratio of window sums (U_e = w_e/n_e, Sec. 2.1),
        mean potential, mean ion flux to the powered electrode, and J0 as the mean over whole
        periods of max |J| (Table "tab:plasmaparameters" quantities)."""
        d = self.d
        nn = self.cfg.n_cells + 1
        V = np.full(nn, d.dx)
        V[0] = V[-1] = 0.5 * d.dx
        N = max(self.n_samples, 1)
        with np.errstate(invalid="ignore", divide="ignore"):
            mean_e = self.m_energy / self.m_dens[ELECTRON]
        window_s = self.n_window_steps * self.cfg.dt_s
        return dict(
            n_e=d.W * self.m_dens[ELECTRON] / (V * N),
            n_i=d.W * self.m_dens[ION] / (V * N),
            mean_energy_e=np.where(self.m_dens[ELECTRON] > 0, mean_e, np.nan),
            flux_i=d.W * self.m_flux / (V * N),
            phi=self.m_phi / N,
            n_samples=self.n_samples,
            window_s=window_s,
            flux_i_powered=(d.W * self.absorbed_window[ION, 0] / window_s) if window_s > 0 else np.nan,
            J0=(self.J_max_sum / self.n_periods) if self.n_periods else np.nan,
            absorbed=self.absorbed_window.copy(),
        )
