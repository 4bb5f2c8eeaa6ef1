"""Host logic of the warm start (no GPU): the steady-state criterion on synthetic period
sequences, and the network's input/output encoding."""
import numpy as np

from paper_1608_04601_amd import warmstart as WS


def _prof(level, rng=None, noise=0.0):
    z = np.linspace(0.0, 1.0, WS.N_POINTS)
    base = np.array([np.sin(np.pi * z) + 0.1, np.sin(np.pi * z) + 0.2, 3.0 + z, 100.0 * z, z - 0.5])
    p = base * level
    if rng is not None:
        p = p * (1.0 + noise * rng.normal(size=p.shape))
    return p


def test_exponential_relaxation_is_detected_when_the_windows_agree():
    rng = np.random.default_rng(0)
    tau = 50.0
    det = WS.SteadyState()
    for c in range(1000):
        level = 2.0 - np.exp(-c / tau)
        det.add(_prof(level, rng, 1e-3), created=1000.0, absorbed=1000.0 * (1.0 + 0.001 * rng.normal()))
        if det.done():
            break
    # two consecutive 20-period means differ by < 1 % once 20 tau' e^{-c/tau} / level < 1 %
    # (a relative change of ~ (20/tau) e^{-c/tau} / 2); that happens near c = tau ln(20) ~ 150
    assert det.steady_at is not None and 120 <= det.steady_at <= 200, det.steady_at
    assert det.done() and det.periods == det.steady_at + det.W


def test_ion_balance_blocks_detection():
    det = WS.SteadyState()
    for c in range(200):
        det.add(_prof(1.0), created=1000.0, absorbed=1050.0)   # 5 % imbalance
    assert det.steady_at is None
    det2 = WS.SteadyState()
    for c in range(200):
        det2.add(_prof(1.0), created=1000.0, absorbed=1020.0)  # 2 %: inside 3 %
    assert det2.steady_at == 40


def test_no_decision_before_two_windows():
    det = WS.SteadyState()
    for c in range(39):
        assert not det.add(_prof(1.0), 10.0, 10.0)
    assert det.add(_prof(1.0), 10.0, 10.0)


def test_a_drifting_quantity_blocks_detection():
    det = WS.SteadyState()
    for c in range(300):
        p = _prof(1.0)
        p[4] += 0.002 * c   # flux keeps drifting: the window means differ by 4e-2 of its max
        det.add(p, 10.0, 10.0)
    assert det.steady_at is None


def test_encoding_round_trip():
    rng = np.random.default_rng(1)
    params = np.stack([rng.uniform(10, 80, 5), rng.uniform(100, 400, 5), rng.uniform(0.02, 0.03, 5),
                       rng.integers(0, 2, 5)], axis=1).astype(float)
    X = WS.encode_inputs(params)
    assert X.shape == (5, 4) and np.all(np.abs(X) <= 1.0 + 1e-6)
    prof = np.abs(rng.normal(size=(5, 5, WS.N_POINTS))) * np.array([1e16, 1e16, 3, 100, 1e19])[None, :, None]
    prof[:, 0, 0] = 0.0   # below the density floor
    back = WS.from_targets(params, WS.to_targets(params, prof))
    expect = prof.copy()
    expect[:, 0, 0] = WS.DENSITY_FLOOR
    np.testing.assert_allclose(back, expect, rtol=1e-12, atol=0)


def test_profile_change_is_relative_rms():
    a = np.ones((5, 10))
    b = a.copy()
    b[2] *= 1.05
    ch = WS.profile_change(a, b)
    np.testing.assert_allclose(ch, [0, 0, 0.05 / 1.05, 0, 0], rtol=1e-12)


def test_large_periodic_weight_matches_the_stored_steady_states():
    """The large discharge's periodic-state weight: with the stored argon steady states
    nearest 80 Pa, 300 V, 3 cm (mean n_e over the gap), the periodic state holds about
    2.5e7 particles per species."""
    import workloads as W
    d = W.large_argon_periodic()
    weight = d.n_init_m3 * d.gap_m / d.n_super[0]
    data = np.load(WS.DATA_PATH)
    P, prof = data["params"], data["profiles"]
    argon = (P[:, 3] == 0) & ~data["extinct"]
    dist = ((P[:, 0] - 80.0) / 70.0) ** 2 + ((P[:, 1] - 300.0) / 300.0) ** 2 + ((P[:, 2] - 0.03) / 0.01) ** 2
    near = np.argsort(np.where(argon, dist, np.inf))[:3]
    n_mean = np.mean([np.mean(prof[k, 0]) for k in near])   # stored n_e in m^-3
    count = n_mean * d.gap_m / weight
    assert 1.5e7 <= count <= 3.5e7, count
    assert d.capacity[0] >= 1.5 * 2.5e7 and d.n_cells == 4096


def test_training_data_concatenates_the_stored_draws(tmp_path):
    a = dict(params=np.zeros((2, 4)), profiles=np.zeros((2, 5, WS.N_POINTS)), extinct=np.array([False, True]))
    b = dict(params=np.ones((3, 4)), profiles=np.ones((3, 5, WS.N_POINTS)), extinct=np.array([False] * 3))
    pa, pb = str(tmp_path / "a.npz"), str(tmp_path / "b.npz")
    np.savez(pa, **a)
    np.savez(pb, **b)
    d = WS.load_data([pa, str(tmp_path / "missing.npz"), pb])
    assert d["params"].shape == (5, 4) and d["profiles"].shape == (5, 5, WS.N_POINTS)
    assert d["extinct"].tolist() == [False, True, False, False, False]
    assert np.all(d["params"][2:] == 1.0)
    full = WS.load_data()
    assert len(full["params"]) >= 128 and full["profiles"].shape[1:] == (5, WS.N_POINTS)


def test_training_uses_only_steady_states():
    """Only draws that met the steady-state criterion are training targets: extinct draws
    and draws still drifting at the period limit (steady_at = -1) are left out."""
    d = dict(extinct=np.array([False, True, False, False]), steady_at=np.array([120, 300, -1, 0]))
    assert WS.training_mask(d).tolist() == [True, False, False, True]
    full = WS.load_data()
    m = WS.training_mask(full)
    assert np.all(full["steady_at"][m] >= 0) and not np.any(full["extinct"][m])
    assert m.sum() < (~full["extinct"]).sum()   # some stored draws were still drifting


def test_summary_counts_runs_that_are_not_steady():
    """Runs that never met the criterion count with the periods they ran (the limit, or what
    a time limit allowed); rows without that record count with the limit."""
    def row(c, w, ran=None, extinct=False):
        r = dict(cold_steady_at=c, warm_steady_at=w, extinct=extinct, warm_vs_cold=[0.01] * 5,
                 prediction_vs_cold=[0.02] * 5)
        if ran is not None:
            r["periods_run"] = ran
        return r
    rows = [row(400, 100), row(None, 80, ran=(1500, 100)), row(None, None), row(300, None, ran=(320, 1500)),
            row(200, 50, extinct=True)]
    sm = WS.summarize(rows, 1500)
    assert sm["discharges"] == 5 and sm["extinct"] == 1 and sm["steady_both"] == 1
    assert sm["cold_periods_mean"] == (400 + 1500 + 1500 + 300) / 4
    assert sm["warm_periods_mean"] == (100 + 80 + 1500 + 1500) / 4
    assert sm["cold_not_steady"] == 2 and sm["warm_not_steady"] == 2
    assert sm["warm_faster"] == 2   # a warm run that is not steady is never the faster one
    big = WS.summarize([row(None, 212, ran=(1246, 232))], 6000)
    assert big["cold_periods_mean"] == 1246 and big["warm_faster"] == 1
