"""Pins of the oracle's initial load, process-selection probabilities, discharge current
and moment normalisation (Sec. 2.2 initial values and current; Sec. 2.5 null collisions;
Table "tab:plasmaparameters" quantities)."""
import numpy as np
from scipy import stats

import workloads as W
from oracle import Oracle, xsec
from oracle.constants import E0, EPS0, ME


def test_load_uniform_maxwellian():
    cfg = W.small_argon(n_super=50_000, seed=3)
    o = Oracle(cfg)
    for s, T in ((0, cfg.te_init_eV), (1, cfg.ti_init_eV)):
        S = o.sp[s]
        assert np.array_equal(S.id, np.arange(50_000)) and S.next_id == 50_000
        assert np.all((S.x > 0) & (S.x < cfg.gap_m))
        assert stats.kstest(S.x / cfg.gap_m, "uniform").pvalue > 1e-4
        sig = np.sqrt(E0 * T / o.d.m[s])
        for c in range(3):
            assert stats.kstest(S.v[:, c] / sig, "norm").pvalue > 1e-4
    # electrons and ions are drawn independently
    assert abs(np.corrcoef(o.sp[0].x, o.sp[1].x)[0, 1]) < 0.02


def test_selection_probabilities_per_process():
    """Monoenergetic electrons: P(process j | candidate) = nu_j(eps)/nu_max, null otherwise."""
    procs = W.argon_like(100.0, 100.0, 0.1, excitation_sigma=4e-20)
    cfg = W.Discharge(name="t", gap_m=1.0, pressure_Pa=20.0, gas_temperature_K=300.0, gas_mass_amu=W.AMU_AR,
                      rf_voltage_V=0.0, rf_frequency_Hz=13.56e6, dt_s=1e-10, n_cells=16, n_init_m3=1e15,
                      te_init_eV=2.0, ti_init_eV=0.026, n_super=(10, 10), capacity=(10, 10), seed=4,
                      processes=procs, sort_every=0, moments_every=1)
    o = Oracle(cfg, load=False, fixed_field=np.zeros(17))
    eps = 40.0
    g = np.sqrt(2 * E0 * eps / ME)
    N = 300_000
    rng = np.random.default_rng(0)
    u = rng.normal(size=(N, 3))
    v = g * u / np.linalg.norm(u, axis=1, keepdims=True)
    st = dict(x=np.full(N, 0.5), vx=v[:, 0], vy=v[:, 1], vz=v[:, 2], id=np.arange(N), next_id=N)
    empty = dict(x=np.zeros(0), vx=np.zeros(0), vy=np.zeros(0), vz=np.zeros(0), id=np.zeros(0), next_id=0)
    o.set_state(0, [st, empty])
    o.step()
    rec = o.last["mcc0"]
    nc = len(rec["candidates"])
    assert abs(nc - N * o.d.T[0] / 2 ** 24) < 5 * np.sqrt(N * 0.25)
    for j in range(3):
        nu_j = o.d.n_gas * xsec.sigma_lookup(procs[j], np.array([eps]))[0] * g
        p = nu_j / o.d.numax[0]
        k = int((rec["selected"] == j).sum())
        assert abs(k - nc * p) < 5 * np.sqrt(nc * p * (1 - p)) + 1, (j, k, nc * p)


def test_current_continuity_between_electrodes():
    """The current at z = 0, eps0 dE_0/dt + e0(Gamma_i - Gamma_e)(0), equals the one at z = d:
    the boundary fields obey Gauss's law and births are neutral, so total current is conserved."""
    cfg = W.small_argon(n_super=4000, seed=2)
    o = Oracle(cfg)
    dt, Wt = cfg.dt_s, o.d.W
    for _ in range(300):
        EN_old = o.E[-1]
        o.step()
        ab = o.last["absorbed"]
        J_d = EPS0 * (o.E[-1] - EN_old) / dt + E0 * Wt * (ab[1, 1] - ab[0, 1]) / dt
        scale = abs(o.J) + abs(J_d) + E0 * Wt / dt
        assert abs(o.J - J_d) < 1e-9 * scale


def test_moments_of_uniform_state():
    """A fresh uniform load sampled once: n ~ n_init at every node (half volume at the
    electrodes), <eps_e> ~ 3/2 k T_e, ion flux ~ 0, phi mean = phi."""
    cfg = W.small_argon(n_super=400_000, seed=1).replace(processes=(), rf_voltage_V=0.0, dt_s=1e-13)
    o = Oracle(cfg, fixed_field=np.zeros(cfg.n_cells + 1))
    o.step()
    m = o.moments()
    assert m["n_samples"] == 1
    for key in ("n_e", "n_i"):
        rel = m[key] / cfg.n_init_m3
        assert abs(rel[1:-1].mean() - 1) < 0.01
        assert abs(rel[[0, -1]].mean() - 1) < 0.1
    assert abs(np.nanmean(m["mean_energy_e"][1:-1]) / (1.5 * cfg.te_init_eV) - 1) < 0.01
    vth_i = np.sqrt(E0 * cfg.ti_init_eV / o.d.M)
    assert np.abs(m["flux_i"][1:-1]).mean() < 0.1 * cfg.n_init_m3 * vth_i
    assert np.allclose(m["phi"], o.phi)


def test_J0_is_mean_of_period_maxima():
    cfg = W.small_argon(n_super=2000, seed=5).replace(dt_s=1.0 / (13.56e6 * 40))
    o = Oracle(cfg)
    Js = []
    for _ in range(3 * 40):
        o.step()
        Js.append(abs(o.J))
    m = o.moments()
    Js = np.array(Js).reshape(3, 40)
    assert np.isclose(m["J0"], Js.max(axis=1).mean(), rtol=1e-14)
    assert m["n_samples"] == 120 and np.isclose(m["window_s"], 120 * cfg.dt_s)


# ---------------------------------------------------------------------------------------
# Ion flux profile and mean ion flux to the powered electrode (Sec. 2.2: the current uses
# Gamma_i(0, t); Table "tab:plasmaparameters": Gamma_i^avg).  Both pins are closed forms
# on hand-placed particles, and each is shown to reject the plausible mistakes of the
# moment formulas (a dropped weight, the full node volume at the electrodes, the wrong
# species' v_x, v_x before the completing kick, counts from the wrong electrode or species).
# ---------------------------------------------------------------------------------------
def _lattice(n_cells, dx, per_cell):
    """per_cell particles per cell at offsets (k + 1/2)/per_cell: every node's CIC sum is
    exactly per_cell inside and per_cell/2 at the electrodes (the hat function's sum over a
    lattice of spacing 1/per_cell is per_cell for any shift)."""
    t = (np.arange(n_cells * per_cell) + 0.5) / per_cell
    return t * dx


def _drift_case(n_cells=32, per_cell=64, v_d=2.0e3, v_de=-7.0e3, a_dt=2.0e3):
    """Ions with v_x = v_d, electrons with v_x = v_de, a uniform external field that
    changes an ion's v_x by a_dt per step, no collisions.  Returns (cfg, oracle, expected
    density, expected ion v_x after the step)."""
    from oracle.constants import AMU
    gap = 0.02
    dt = 1.0e-12
    dx = gap / n_cells
    M = W.AMU_AR * AMU
    E_c = a_dt * M / (E0 * dt)                 # q E / M dt = a_dt for ions
    N = n_cells * per_cell
    cfg = W.small_argon(n_super=N, seed=0).replace(processes=(), rf_voltage_V=0.0, dt_s=dt, n_cells=n_cells,
                                                   gap_m=gap, n_super=(N, N), capacity=(N, N))
    o = Oracle(cfg, load=False, fixed_field=np.full(n_cells + 1, E_c))
    x = _lattice(n_cells, dx, per_cell)
    zeros = np.zeros(N)
    elec = dict(x=x.copy(), vx=np.full(N, v_de), vy=zeros, vz=zeros, id=np.arange(N), next_id=N)
    ion = dict(x=x.copy(), vx=np.full(N, v_d), vy=zeros, vz=zeros, id=np.arange(N), next_id=N)
    o.set_state(0, [elec, ion])
    n_expected = o.d.W * per_cell / dx          # one particle's W per lattice spacing dx/per_cell
    return cfg, o, n_expected, v_d + a_dt


def _flux_pin_holds(m, n_expected, v_expected, dx_shift_rel):
    """The drift-flux closed form: n_i equal to the lattice density at every node (to the
    shift of one drift step), and Gamma_i = n_i v_x at every node to rounding."""
    n_i, flux = m["n_i"], m["flux_i"]
    if not np.all(np.abs(n_i / n_expected - 1.0) <= 2.0 * dx_shift_rel + 1e-12):
        return False
    return bool(np.all(np.abs(flux - n_i * v_expected) <= 1e-12 * np.abs(n_i * v_expected)))


def test_ion_flux_of_uniform_drift():
    cfg, o, n_exp, v_exp = _drift_case()
    o.step()
    m = o.moments()
    assert m["n_samples"] == 1
    # one step moves every particle by at most v dt / dx of a cell; the end nodes see it
    shift = 1.1 * max(abs(v_exp), 7.0e3) * cfg.dt_s / (cfg.gap_m / cfg.n_cells)
    assert _flux_pin_holds(m, n_exp, v_exp, shift)
    assert np.allclose(m["flux_i"], n_exp * v_exp, rtol=2.0 * shift + 1e-12)


class _NoWeightFlux(Oracle):
    def moments(self):
        m = super().moments()
        m["flux_i"] = m["flux_i"] / self.d.W
        return m


class _FullVolumeFlux(Oracle):
    def moments(self):
        m = super().moments()
        f = m["flux_i"].copy()
        f[[0, -1]] *= 0.5                           # dx instead of dx/2 at the electrodes
        m["flux_i"] = f
        return m


class _ElectronVxFlux(Oracle):
    def _accumulate(self, absorbed):
        super()._accumulate(absorbed)
        if self.n % self.cfg.moments_every == 0:   # replace this sample's ion v_x by the electrons'
            from oracle import field
            d = self.d
            Si, Se = self.sp[1], self.sp[0]
            self.m_flux -= field.deposit(Si.x, Si.v[:, 0], d.dx, self.cfg.n_cells)
            self.m_flux += field.deposit(Se.x, Se.v[:, 0], d.dx, self.cfg.n_cells)


class _HalfKickFlux(Oracle):
    """Samples v_x before the completing half kick (the uniform field's a dt / 2 missing)."""
    def _accumulate(self, absorbed):
        super()._accumulate(absorbed)
        if self.n % self.cfg.moments_every == 0:
            from oracle import field
            d = self.d
            Si = self.sp[1]
            a = d.q[1] / d.m[1] * self._gather_E(Si.x)
            self.m_flux -= field.deposit(Si.x, 0.5 * a * self.cfg.dt_s, d.dx, self.cfg.n_cells)


def test_ion_flux_pin_rejects_planted_mistakes():
    for cls in (_NoWeightFlux, _FullVolumeFlux, _ElectronVxFlux, _HalfKickFlux):
        cfg, o, n_exp, v_exp = _drift_case()
        o.__class__ = cls
        o.step()
        shift = 1.1 * 7.0e3 * cfg.dt_s / (cfg.gap_m / cfg.n_cells)
        assert not _flux_pin_holds(o.moments(), n_exp, v_exp, shift), cls.__name__


def _powered_case(K=37, K_decoy=23, K_e=11, steps=3):
    """K ions placed to reach z = 0 in the first step, K_decoy ions that reach z = d, K_e
    electrons that reach z = 0, and a few ions that stay; no field, no collisions."""
    gap, n_cells, dt = 0.02, 16, 1.0e-10
    N = K + K_decoy + 5
    cfg = W.small_argon(n_super=max(K_e, 1), seed=0).replace(processes=(), rf_voltage_V=0.0, dt_s=dt,
                                                             n_cells=n_cells, gap_m=gap, n_super=(max(K_e, 1), N),
                                                             capacity=(max(K_e, 1), N))
    o = Oracle(cfg, load=False, fixed_field=np.zeros(n_cells + 1))
    rng = np.random.default_rng(7)
    v_far = 1.0e6                                   # 100 um per step: every crosser is out in one step
    x_i = np.concatenate([rng.uniform(1e-6, 5e-5, K), gap - rng.uniform(1e-6, 5e-5, K_decoy),
                          rng.uniform(0.3 * gap, 0.7 * gap, 5)])
    vx_i = np.concatenate([np.full(K, -v_far), np.full(K_decoy, v_far), np.zeros(5)])
    x_e = rng.uniform(1e-6, 5e-5, K_e)
    zi, ze = np.zeros(N), np.zeros(K_e)
    o.set_state(0, [dict(x=x_e, vx=np.full(K_e, -v_far), vy=ze, vz=ze, id=np.arange(K_e), next_id=K_e),
                    dict(x=x_i, vx=vx_i, vy=zi, vz=zi, id=np.arange(N), next_id=N)])
    for _ in range(steps):
        o.step()
    return o, K, steps


def _powered_pin_holds(o, K, steps):
    m = o.moments()
    return m["flux_i_powered"] == o.d.W * K / (steps * o.cfg.dt_s)


def test_ion_flux_to_powered_electrode_counts():
    o, K, steps = _powered_case()
    m = o.moments()
    assert np.isclose(m["window_s"], steps * o.cfg.dt_s, rtol=1e-15)
    assert m["absorbed"][1, 0] == K and m["absorbed"][1, 1] == 23 and m["absorbed"][0, 0] == 11
    assert _powered_pin_holds(o, K, steps)


class _FarElectrodeFlux(Oracle):
    def moments(self):
        m = super().moments()
        m["flux_i_powered"] = self.d.W * self.absorbed_window[1, 1] / m["window_s"]
        return m


class _ElectronCountFlux(Oracle):
    def moments(self):
        m = super().moments()
        m["flux_i_powered"] = self.d.W * self.absorbed_window[0, 0] / m["window_s"]
        return m


class _NoWeightPowered(Oracle):
    def moments(self):
        m = super().moments()
        m["flux_i_powered"] = self.absorbed_window[1, 0] / m["window_s"]
        return m


def test_powered_flux_pin_rejects_planted_mistakes():
    for cls in (_FarElectrodeFlux, _ElectronCountFlux, _NoWeightPowered):
        o, K, steps = _powered_case()
        o.__class__ = cls
        assert not _powered_pin_holds(o, K, steps), cls.__name__
