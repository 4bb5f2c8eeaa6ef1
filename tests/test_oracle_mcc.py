"""Pins of the oracle's null-collision MCC (Sec. 2.5; Table "tab:reactions")."""
import numpy as np
import pytest
from scipy import special, stats

import workloads as W
from oracle import Oracle, xsec
from oracle.constants import AMU, E0, KB, ME


def _cfg(procs, **kw):
    base = dict(name="t", gap_m=1.0, pressure_Pa=20.0, gas_temperature_K=300.0, gas_mass_amu=W.AMU_AR,
                rf_voltage_V=0.0, rf_frequency_Hz=13.56e6, dt_s=1e-10, n_cells=16, n_init_m3=1e15,
                te_init_eV=2.0, ti_init_eV=0.026, n_super=(100, 100), capacity=(10 ** 7, 10 ** 7), seed=11,
                processes=tuple(procs), sort_every=0, moments_every=1)
    base.update(kw)
    return W.Discharge(**base)


def _state(x, v, ids=None, next_id=None):
    v = np.asarray(v, float).reshape(-1, 3)
    ids = np.arange(len(x)) if ids is None else ids
    return dict(x=np.asarray(x, float), vx=v[:, 0], vy=v[:, 1], vz=v[:, 2], id=ids,
                next_id=len(x) if next_id is None else next_id)


def _empty():
    return _state(np.zeros(0), np.zeros((0, 3)))


def _iso(n, speed, rng):
    u = rng.normal(size=(n, 3))
    return speed * u / np.linalg.norm(u, axis=1, keepdims=True)


def test_sigma_lookup_rules():
    tab = np.array([0.0, 1.0, 3.0, 3.0, 2.0])
    p = W.Process(W.E_EXCITATION, W.FRAME_LAB, 1.5, 1.0, 0.0, tab)
    eps = np.array([0.0, 1.49, 1.5, 1.75, 2.0, 3.5, 4.0, 100.0])
    got = xsec.sigma_lookup(p, eps)
    assert np.allclose(got, [0, 0, 2.0, 2.5, 3.0, 2.5, 2.0, 2.0])
    q = W.Process(W.I_BACKWARD, W.FRAME_LAB, 0.0, 1.0, 2.5, tab)
    assert np.allclose(xsec.sigma_lookup(q, np.array([0.0, 1.0, 2.5, 3.0])), [3.0, 3.0, 3.0, 3.0])


def test_numax_closed_form_and_brute_force():
    M = W.AMU_AR * AMU
    n_gas = 4.8e21
    const = W.Process(W.E_ELASTIC, W.FRAME_LAB, 0.0, 0.5, 0.0, W.constant_table(1e-19, 200.0, 0.5))
    nm = xsec.nu_max([const], ME, M, n_gas)
    assert np.isclose(nm, n_gas * 1e-19 * np.sqrt(2 * E0 * 200.0 / ME), rtol=1e-13)
    # decreasing table: interior maximum of (a + b eps) sqrt(eps) inside a segment
    tab = np.array([5.0, 4.0, 1.0, 0.5, 0.4]) * 1e-20
    dec = W.Process(W.E_ELASTIC, W.FRAME_LAB, 0.0, 2.0, 0.0, tab)
    procs = [dec] + list(W.argon_like(8.0, 8.0, 0.25)[1:3])
    nm = xsec.nu_max(procs, ME, M, n_gas)
    eps = np.linspace(0, 8.0, 2_000_001)
    brute = n_gas * sum(xsec.sigma_lookup(p, eps) for p in procs) * np.sqrt(2 * E0 * eps / ME)
    assert brute.max() <= nm * (1 + 1e-12)
    assert brute.max() >= nm * (1 - 1e-9)
    # CM frame: the CM energy is M/(m+M) of the lab energy
    cm = W.Process(W.I_BACKWARD, W.FRAME_CM, 0.0, 0.1, 0.0, W.constant_table(5e-19, 10.0, 0.1))
    nm = xsec.nu_max([cm], M, M, n_gas)
    assert np.isclose(nm, n_gas * 5e-19 * np.sqrt(2 * E0 * 20.0 / M), rtol=1e-13)


def test_free_flight_law():
    """Electrons at the table top with one constant process have nu = nu_max: the candidate
    probability is T/2^24 ~ 1 - exp(-nu dt), every candidate collides, and the never-collided
    fraction after k steps is (1 - T/2^24)^k."""
    eps0 = 10.0
    proc = W.Process(W.E_ELASTIC, W.FRAME_LAB, 0.0, 0.05, 0.0, W.constant_table(1e-19, eps0, 0.05))
    cfg = _cfg([proc], dt_s=2e-10)
    o = Oracle(cfg, load=False, fixed_field=np.zeros(17))
    g0 = np.sqrt(2 * E0 * eps0 / ME)
    nu = o.d.n_gas * 1e-19 * g0
    assert np.isclose(o.d.numax[0], nu, rtol=1e-13)
    p = -np.expm1(-nu * cfg.dt_s)
    assert o.d.T[0] == round(p * 2 ** 24)
    N, K = 40_000, 6
    rng = np.random.default_rng(5)
    o.set_state(0, [_state(np.full(N, 0.5), _iso(N, g0, rng)), _empty()])
    never = np.ones(N, bool)
    ids_all = np.arange(N)
    for _ in range(K):
        o.step()
        rec = o.last["mcc0"]
        fresh = never[rec["candidates"].astype(np.int64)]
        # at the table top R < c = nu_max holds for every candidate (elastic losses then
        # lower nu below nu_max, so later collisions may be null)
        assert fresh.any() and np.all(rec["selected"][fresh] == 0)
        never[np.isin(ids_all, rec["candidates"])] = False
    q = (1 - o.d.T[0] / 2 ** 24) ** K
    z = (never.sum() - N * q) / np.sqrt(N * q * (1 - q))
    assert abs(z) < 5, z
    assert abs(q - np.exp(-nu * K * cfg.dt_s)) < 1e-6


def test_ion_collision_rate_maxwellian_target():
    """Constant sigma: the real-collision rate of an ion of speed v in the thermal gas is
    n sigma <g>, <g> = a[(s + 1/(2s)) erf(s) + exp(-s^2)/sqrt(pi)], a = sqrt(2kT/M), s = v/a."""
    proc = W.Process(W.I_BACKWARD, W.FRAME_LAB, 0.0, 0.1, 0.0, W.constant_table(5e-19, 2.0, 0.1))
    cfg = _cfg([proc], dt_s=2e-7)
    o = Oracle(cfg, load=False, fixed_field=np.zeros(17))
    M = o.d.M
    a = np.sqrt(2 * KB * 300.0 / M)
    rng = np.random.default_rng(6)
    for s_ratio in (0.3, 1.0, 3.0):
        v = s_ratio * a
        N = 200_000
        o.set_state(0, [_empty(), _state(np.full(N, 0.5), _iso(N, v, rng))])
        o.step()
        sel = o.last["mcc1"]["selected"]
        gmean = a * ((s_ratio + 1 / (2 * s_ratio)) * special.erf(s_ratio) + np.exp(-s_ratio ** 2) / np.sqrt(np.pi))
        p = (o.d.T[1] / 2 ** 24) * o.d.n_gas * 5e-19 * gmean / o.d.numax[1]
        hits = int((sel >= 0).sum())
        z = (hits - N * p) / np.sqrt(N * p * (1 - p))
        assert abs(z) < 5, (s_ratio, z)


def _collisional_oracle(seed=3):
    procs = (
        W.Process(W.E_ELASTIC, W.FRAME_LAB, 0.0, 0.1, 0.0, W.constant_table(1e-19, 60.0, 0.1)),
        W.Process(W.E_EXCITATION, W.FRAME_LAB, 11.5, 0.1, 0.0, W.ramp_table(11.5, 5e-20, 60.0, 0.1)),
        W.Process(W.E_IONIZATION, W.FRAME_LAB, 15.8, 0.1, 0.0, W.ramp_table(15.8, 8e-20, 60.0, 0.1)),
        W.Process(W.I_ISOTROPIC, W.FRAME_CM, 0.0, 0.1, 0.0, W.constant_table(3e-19, 60.0, 0.1)),
        W.Process(W.I_BACKWARD, W.FRAME_LAB, 0.0, 0.1, 0.1, W.constant_table(5e-19, 60.0, 0.1)),
    )
    cfg = _cfg(procs, dt_s=1e-10, seed=seed)
    o = Oracle(cfg, load=False, fixed_field=np.zeros(17))
    rng = np.random.default_rng(seed)
    N = 30_000
    ve = _iso(N, 1.0, rng) * np.sqrt(2 * E0 * rng.uniform(0, 55, N) / ME)[:, None]
    vi = _iso(N, 1.0, rng) * np.sqrt(2 * E0 * rng.uniform(0, 30, N) / o.d.M)[:, None]
    o.set_state(0, [_state(rng.uniform(0.3, 0.7, N), ve), _state(rng.uniform(0.3, 0.7, N), vi)])
    return o


def test_collision_invariants():
    o = _collisional_oracle()
    M, m_e = o.d.M, ME
    seen = set()
    for _ in range(3):
        before_next = [o.sp[0].next_id, o.sp[1].next_id]
        o.step()
        for s, m in ((0, m_e), (1, M)):
            rec = o.last[f"mcc{s}"]
            sel = rec["selected"]
            vb, va, vt = rec["v_before"], rec["v_after"], rec["v_target"]
            for j, p in enumerate(o.procs):
                k = sel == j
                if not k.any():
                    continue
                seen.add(p.kind)
                eb = 0.5 * m * (vb[k] ** 2).sum(1) / E0
                ea = 0.5 * m * (va[k] ** 2).sum(1) / E0
                if p.kind in (W.E_ELASTIC, W.I_ISOTROPIC):
                    # momentum and energy of the (particle, atom) pair are conserved
                    vt_after = (m * vb[k] + M * vt[k] - m * va[k]) / M
                    e_pair_b = 0.5 * m * (vb[k] ** 2).sum(1) + 0.5 * M * (vt[k] ** 2).sum(1)
                    e_pair_a = 0.5 * m * (va[k] ** 2).sum(1) + 0.5 * M * (vt_after ** 2).sum(1)
                    assert np.allclose(e_pair_a, e_pair_b, rtol=1e-9)
                    if p.kind == W.E_ELASTIC:
                        assert np.all(ea <= eb * (1 + 1e-12))
                elif p.kind == W.E_EXCITATION:
                    assert np.allclose(ea, eb - p.threshold_eV, rtol=1e-9, atol=1e-9)
                elif p.kind == W.I_BACKWARD:
                    assert np.array_equal(va[k], vt[k])
                elif p.kind == W.E_IONIZATION:
                    births = o.last["births"]
                    cand = rec["candidates"][k]
                    assert np.array_equal(np.sort(cand), births["parent"])
                    # children: ids in ascending parent order; same energy as the parent
                    Se = o.sp[0]
                    order = np.argsort(cand)
                    child_ids = before_next[0] + np.arange(len(cand))
                    slot = {int(i): n for n, i in enumerate(Se.id)}
                    for r, idx in enumerate(order):
                        ci = slot[int(child_ids[r])]
                        pi = slot[int(cand[idx])]
                        e_child = 0.5 * m_e * (Se.v[ci] ** 2).sum() / E0
                        assert np.isclose(e_child, ea[idx], rtol=1e-12)
                        assert np.isclose(eb[idx], p.threshold_eV + ea[idx] + e_child, rtol=1e-9)
                        assert Se.x[ci] == Se.x[pi]
                        ion = o.sp[1]
                        ii = int(np.nonzero(ion.id == before_next[1] + r)[0][0])
                        assert ion.x[ii] == Se.x[pi]
    assert seen == {W.E_ELASTIC, W.E_EXCITATION, W.E_IONIZATION, W.I_ISOTROPIC, W.I_BACKWARD}


@pytest.mark.parametrize("kind", [W.I_BACKWARD, W.I_ISOTROPIC])
def test_maxwellian_relaxation(kind):
    """Ions started monoenergetic (1 eV) relax under charge exchange or isotropic elastic
    collisions with the 300 K gas to the gas Maxwellian."""
    proc = W.Process(kind, W.FRAME_LAB, 0.0, 0.01, 0.0, W.constant_table(5e-19, 1.2, 0.01))
    cfg = _cfg([proc], gap_m=100.0, dt_s=2e-7)
    o = Oracle(cfg, load=False, fixed_field=np.zeros(17))
    M = o.d.M
    rng = np.random.default_rng(8)
    N = 40_000
    o.set_state(0, [_empty(), _state(np.full(N, 50.0), _iso(N, np.sqrt(2 * E0 * 1.0 / M), rng))])
    for _ in range(250 if kind == W.I_BACKWARD else 500):
        o.step()
    v = o.sp[1].v
    assert len(v) == N
    kT = KB * 300.0
    mean_e = 0.5 * M * (v ** 2).sum(1).mean()
    assert abs(mean_e / (1.5 * kT) - 1) < 4 * np.sqrt(2 / 3) / np.sqrt(N) + 2e-3
    for c in range(3):
        z = v[:, c] / np.sqrt(kT / M)
        assert abs(z.var() - 1) < 0.03
        assert abs(stats.kurtosis(z, fisher=False) - 3) < 0.15
        assert stats.kstest(z, "norm").pvalue > 1e-4
