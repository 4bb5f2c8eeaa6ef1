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
