"""Pins of the oracle's velocity-Verlet push (Sec. 2.5) and of its whole-step
bookkeeping (charge conservation, Gauss's law, absorption counts)."""
import numpy as np
import pytest

import workloads as W
from oracle import Oracle
from oracle.constants import E0, EPS0, ME


def _cfg(**kw):
    base = dict(name="t", gap_m=0.02, pressure_Pa=20.0, gas_temperature_K=300.0, gas_mass_amu=W.AMU_AR,
                rf_voltage_V=0.0, rf_frequency_Hz=13.56e6, dt_s=1e-10, n_cells=64, n_init_m3=1e15,
                te_init_eV=2.0, ti_init_eV=0.026, n_super=(100, 100), capacity=(1000, 1000), seed=0,
                processes=(), sort_every=0, moments_every=1)
    base.update(kw)
    return W.Discharge(**base)


def _state(x, v, ids=None):
    x = np.asarray(x, float)
    v = np.asarray(v, float).reshape(-1, 3)
    ids = np.arange(len(x)) if ids is None else ids
    return dict(x=x, vx=v[:, 0], vy=v[:, 1], vz=v[:, 2], id=ids, next_id=len(x))


def _empty():
    return _state(np.zeros(0), np.zeros((0, 3)))


def test_verlet_constant_field_parabola():
    cfg = _cfg(gap_m=1.0, n_cells=16, dt_s=1e-9)
    Ec = -250.0
    o = Oracle(cfg, load=False, fixed_field=np.full(17, Ec))
    rng = np.random.default_rng(0)
    x0 = rng.uniform(0.4, 0.6, 50)
    v0 = rng.normal(size=(50, 3)) * 1e4
    o.set_state(0, [_state(x0, v0), _empty()])
    a = -E0 / ME * Ec
    for n in range(1, 101):
        o.step()
        st = o.state(0)
        t = n * cfg.dt_s
        assert np.allclose(st["x"], x0 + v0[:, 0] * t + 0.5 * a * t * t, rtol=1e-12, atol=1e-14)
        assert np.allclose(st["vx"], v0[:, 0] + a * t, rtol=1e-12, atol=1e-6)
        assert np.array_equal(st["vy"], v0[:, 1])


@pytest.mark.parametrize("omega_dt", [0.05, 0.3, 1.2])
def test_verlet_harmonic_discrete_map(omega_dt):
    """E = kappa (x - c): x_n - c = A cos(n theta) + B sin(n theta), cos theta = 1 - (w dt)^2/2,
    and v^2 + w^2 (1 - w^2 dt^2/4) (x - c)^2 is conserved exactly."""
    d, nc, dt = 0.02, 64, 1e-10
    c = d / 2
    omega = omega_dt / dt
    kappa = omega ** 2 * ME / E0  # electron: a = -(e/m) kappa (x - c)
    nodes = np.arange(nc + 1) * d / nc
    o = Oracle(_cfg(gap_m=d, n_cells=nc, dt_s=dt), load=False, fixed_field=kappa * (nodes - c))
    rng = np.random.default_rng(1)
    x0 = c + rng.uniform(-0.2, 0.2, 20) * d
    v0 = np.zeros((20, 3))
    v0[:, 0] = rng.uniform(-1, 1, 20) * 0.1 * omega * d
    o.set_state(0, [_state(x0, v0), _empty()])
    theta = np.arccos(1 - omega_dt ** 2 / 2)
    A = x0 - c
    B = v0[:, 0] * dt / np.sin(theta)
    H0 = v0[:, 0] ** 2 + omega ** 2 * (1 - omega_dt ** 2 / 4) * A ** 2
    for n in range(1, 1001):
        o.step()
        if n % 50:
            continue
        st = o.state(0)
        assert st["x"].size == 20
        ref = c + A * np.cos(n * theta) + B * np.sin(n * theta)
        assert np.allclose(st["x"], ref, rtol=0, atol=1e-12 * d)
        H = st["vx"] ** 2 + omega ** 2 * (1 - omega_dt ** 2 / 4) * (st["x"] - c) ** 2
        assert np.allclose(H, H0, rtol=1e-10)


def test_absorption_counts_and_removal():
    # binary fractions make the wall hits exact: ties (x == 0, x == d) are absorbed
    d, dt = 2.0 ** -6, 2.0 ** -30
    cfg = _cfg(gap_m=d, n_cells=16, dt_s=dt)
    o = Oracle(cfg, load=False, fixed_field=np.zeros(17))
    step = 2.0 ** -10
    x = np.array([step, d - step, d / 2, step / 2, d - step / 4])
    v = np.zeros((5, 3))
    v[:, 0] = np.array([-1.0, 1.0, 0.0, -1.0, 0.0]) * step / dt
    o.set_state(0, [_state(x, v), _state(x[:2], v[:2] * 0)])
    o.step()
    ab = o.last["absorbed"]
    assert ab[0, 0] == 2 and ab[0, 1] == 1 and ab[1].sum() == 0
    assert sorted(o.state(0)["id"].tolist()) == [2, 4]


def test_charge_conservation_and_gauss_during_discharge():
    cfg = W.small_argon(n_super=3000)
    o = Oracle(cfg)
    Wt = o.d.W
    for _ in range(60):
        o.step()
        ne, ni = len(o.sp[0].x), len(o.sp[1].x)
        assert np.isclose(o.Q.sum(), E0 * Wt * (ni - ne), rtol=1e-12, atol=1e-12 * E0 * Wt * (ni + ne))
        assert abs(o.sigma0 + o.sigmad + o.Q.sum()) < 1e-12 * np.abs(o.Q).sum() + 1e-30
        # the powered electrode follows V0 sin(2 pi f t_n)
        assert np.isclose(o.phi[0], cfg.rf_voltage_V * np.sin(2 * np.pi * cfg.rf_frequency_Hz * o.n * cfg.dt_s))
        assert o.phi[-1] == 0.0
