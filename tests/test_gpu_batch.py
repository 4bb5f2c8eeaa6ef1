"""Batched discharges through the C ABI: one particle-pass launch per step advances several
independent discharges of different sizes, grids and gases.  Since every random number is
keyed by particle id and the deposit is exact, each discharge of a batch must end bitwise
equal, per id, to the same discharge advanced alone; per-discharge calls between batched
steps must not change that."""
import numpy as np
import pytest

import workloads as W
from gpu_common import log
from paper_1608_04601_amd import binding as B

pytestmark = pytest.mark.gpu


def _members():
    a = W.small_argon(seed=11)
    b = W.small_argon(seed=12, n_super=7_003).replace(n_cells=77, sort_every=7)
    top = 400.0
    c = W.production_helium(seed=13, n_super=15_000).replace(
        n_cells=200, capacity=(60_000, 60_000), dt_s=1.0 / (13.56e6 * 400),
        processes=W.helium_like(top, top))
    return [a, b, c]


def _state(v):
    return [v.particles(0), v.particles(1), v.counters(), v.fields()]


def _same(x, y, tag):
    for s in (0, 1):
        a, b = x[s], y[s]
        ka, kb = np.argsort(a["id"]), np.argsort(b["id"])
        assert np.array_equal(a["id"][ka], b["id"][kb]), (tag, s)
        for key in ("x", "vx", "vy", "vz"):
            assert np.array_equal(a[key][ka], b[key][kb]), (tag, s, key)
    for key in ("step", "n_alive", "next_id", "births_total"):
        assert x[2][key] == y[2][key], (tag, key)
    assert x[2]["collisions"].tolist() == y[2]["collisions"].tolist(), tag
    assert np.array_equal(x[3]["E"], y[3]["E"]), tag
    assert np.array_equal(x[3]["phi"], y[3]["phi"]), tag


def test_batch_equals_solo_runs():
    discs = _members()
    log("batch vs solo: " + ", ".join(f"{d.n_cells}c/{d.n_super[0]}" for d in discs))
    with B.Batch(discs) as bt:
        assert all(bt.blocks(k) >= 2 for k in range(len(bt)))
        bt.step(90)
        bt.sync()
        got = [_state(bt[k]) for k in range(len(bt))]
        mom = [bt[k].moments() for k in range(len(bt))]
    for k, d in enumerate(discs):
        with B.Discharge(d) as solo:
            solo.step(90)
            ref = _state(solo)
            mref = solo.moments()
        _same(got[k], ref, k)
        for key in ("n_e", "n_i", "flux_i", "phi"):   # window sums: FP64 atomics, order may differ
            np.testing.assert_allclose(mom[k][key], mref[key], rtol=1e-12, atol=1e-30)


def test_batch_with_per_discharge_calls_in_between():
    discs = _members()
    with B.Batch(discs) as bt:
        bt.step(25)
        bt[1].counters()          # completes discharge 1 alone: pending states now differ
        bt[2].particles(0)
        bt.step(30)
        got = [_state(bt[k]) for k in range(len(bt))]
    for k, d in enumerate(discs):
        with B.Discharge(d) as solo:
            solo.step(55)
            _same(got[k], _state(solo), k)


def _common_sort_members(sort_every=5):
    return [d.replace(sort_every=sort_every) for d in _members()]


def test_batched_reordering_equals_solo_runs():
    """Every discharge due in the same step: the reordering runs as one launch per stage."""
    discs = _common_sort_members()
    with B.Batch(discs) as bt:
        bt.step(37)
        got = [_state(bt[k]) for k in range(len(bt))]
    for k, d in enumerate(discs):
        with B.Discharge(d) as solo:
            solo.step(37)
            _same(got[k], _state(solo), k)


def test_graph_replays_equal_eager_steps():
    """Steps replayed from a captured graph, with eager steps, queries and synchronisation
    between the replays, against the same batch stepped launch by launch; every replay is
    checked.  Runs of 10 steps keep the reordering phase (every 5 steps), a run of 3 steps
    shifts it and forces a second capture."""
    discs = _common_sort_members()
    with B.Batch(discs) as g, B.Batch(discs) as e:
        g.set_graph(10)
        replays = 0
        for n in (10, 10, 3, 10, 10, 12):
            g.step(n)
            e.step(n)
            replays += n // 10
            g.sync()
            e.sync()
            assert g.graph_launches() == replays
            for k in range(len(discs)):
                _same(_state(g[k]), _state(e[k]), (n, k))
        log(f"graph replays checked: {replays}")


def test_rebalance_keeps_results():
    """Re-splitting the workgroups by the current counts (after a warm load of one member,
    which changes its count several-fold) changes no result."""
    discs = _common_sort_members()
    z = np.linspace(0.0, discs[0].gap_m, 33)
    prof = dict(n_e=3e15 * np.sin(np.pi * z / z[-1]) ** 2 + 1e13, n_i=3e15 * np.sin(np.pi * z / z[-1]) + 1e13,
                mean_energy_e=np.full(33, 3.0), flux_i=np.zeros(33))
    with B.Batch(discs) as bt:
        B.pic_load_profiles(bt[0].h, prof["n_e"], prof["n_i"], prof["mean_energy_e"], prof["flux_i"])
        g0 = bt.blocks(0)
        bt.rebalance()
        assert bt.blocks(0) > g0
        bt.step(12)
        bt.rebalance()
        bt.step(9)
        got = [_state(bt[k]) for k in range(len(bt))]
    for k, d in enumerate(discs):
        with B.Discharge(d) as solo:
            if k == 0:
                B.pic_load_profiles(solo.h, prof["n_e"], prof["n_i"], prof["mean_energy_e"], prof["flux_i"])
            solo.step(21)
            _same(got[k], _state(solo), k)


def test_autotune_choice_is_valid_and_keeps_results():
    """The tuner's trials advance the batch under other launch shapes and reordering
    schedules; the state must still equal, per id, each discharge advanced alone by the
    same number of steps."""
    discs = _common_sort_members()
    with B.Batch(discs) as bt:
        bt.step(3)
        t = bt.autotune(steps_per_trial=8)
        log(f"autotune: {t}")
        assert t["trials"] >= 10 and t["ms_per_step"] > 0
        assert t["threads"] in (256, 512, 1024) and t["rounds"] in (1.0, 2.0, 4.0, 8.0)
        assert t["sort_every"] in (5, 10, 20, 40, 80) and t["electron_order"] in (-1, 0, 1)
        bt.step(7)
        got = [_state(bt[k]) for k in range(len(bt))]
    steps = got[0][2]["step"]
    assert all(g[2]["step"] == steps for g in got) and steps > 10
    for k, d in enumerate(discs):
        with B.Discharge(d) as solo:
            solo.step(steps)
            _same(got[k], _state(solo), k)


def _sweep_members():
    """Three discharges of the sweep's kind (argon-like, T_rf/2000, uneven sizes and grids);
    the middle one has the sweep's shape and is the one checked against the oracle."""
    sw = W.sweep_argon()
    checked = W.sweep_argon(1, seed=5)[0].replace(n_cells=576, n_super=(120_000, 120_000),
                                                  capacity=(480_000, 480_000), name="sweep_checked")
    return [sw[3], checked, sw[7]]


def _member_parity(discs, k, checkpoints):
    """Advance the batch by batched launches; at each checkpoint hand member k's state to the
    FP64 oracle and take one step on both: the drift, deposit and solve in the batched
    advancing launch, the MCC and births in the batched completing launch, with decision
    records on.  Checked as in the single-discharge protocol: fields, per-id positions and
    velocities, candidate sets, process choices outside the margin band,
    ionisation-product ids."""
    from gpu_common import REL_FIELD, compare_decisions, compare_species, oracle_input
    from oracle import Oracle
    disc = discs[k]
    with B.Batch(discs) as bt:
        log(f"batch member parity: member {k} of {len(discs)}, {disc.n_cells} cells, {disc.n_super[0]} per species, "
            f"{bt.blocks(k)} of {sum(bt.blocks(q) for q in range(len(bt)))} workgroups")
        bt.record_decisions(True)
        for n in checkpoints:
            bt.step(n)
            bt.sync()                  # batched completing launch: nothing is left pending
            v = bt[k]
            c0 = v.counters()
            o = Oracle(disc, load=False)
            o.set_state(c0["step"], oracle_input(v, c0))
            bt.step(1)                 # batched advancing launch
            bt.sync()                  # batched completing launch (MCC, births)
            o.step()
            c1 = v.counters()
            f = v.fields()
            assert c1["step"] == c0["step"] + 1
            assert np.max(np.abs(f["E"] - o.E)) <= REL_FIELD * np.abs(o.E).max()
            assert np.max(np.abs(f["phi"] - o.phi)) <= REL_FIELD * max(np.abs(o.phi).max(), disc.rf_voltage_V)
            choice, unsure = {}, [set(), set()]
            for s in (0, 1):
                ch, unsure[s] = compare_decisions(o, s, B.pic_get_decisions(v.h, s), c0["next_id"][s])
                choice.update({(s, i): j for i, j in ch.items()})
            iz = [j for j, p in enumerate(disc.processes) if p.kind == W.E_IONIZATION]
            g_par = {i for (s, i), j in choice.items() if s == 0 and j in iz}
            o_par = set(o.last["births"]["parent"].astype(np.int64).tolist())
            assert (g_par ^ o_par) <= unsure[0]
            same_births = g_par == o_par
            if same_births:
                assert c1["next_id"] == (o.sp[0].next_id, o.sp[1].next_id)
            n_cand = sum(len(o.last[f"mcc{s}"]["candidates"]) for s in (0, 1))
            for s in (0, 1):
                skip = 1 << 62 if same_births else c0["next_id"][s]
                n_cmp = compare_species(o, s, v.particles(s), unsure[s], skip, disc)
                assert n_cmp > 0.99 * len(o.sp[s].x) - len(unsure[s]) - 4
            log(f"  step {c0['step']}->{c1['step']}: {n_cand} candidates, {len(o_par)} births, "
                f"excused choices {len(unsure[0]) + len(unsure[1])}")
        assert v.counters()["numax_violations"] == (0, 0)


def test_batch_member_single_step_parity_against_oracle():
    """A member of sweep shape (576 cells, 1.2e5 particles per species) advanced by batched
    launches in the batch's own launch shape, checked against the oracle after 60 and 121
    steps."""
    _member_parity(_sweep_members(), 1, (60, 60))


def test_full_sweep_member_single_step_parity_against_oracle():
    """The full 64-discharge sweep in the launch shape its benchmark times (the batch's
    default schedule, which its tuner keeps), one member checked against the oracle after 45
    steps, when the uniform starts are ionising hardest; the member with the most particles
    is the one checked."""
    discs = W.sweep_argon()
    k = int(np.argmax([d.n_super[0] for d in discs]))
    _member_parity(discs, k, (45,))


def test_single_discharge_graph_replays_equal_eager_steps():
    """One discharge stepped through pic_set_graph (graphs of 10 steps, reordering every 5)
    against the same discharge launched step by step; eager steps, queries and
    synchronisation between the replays, every replay checked; a run of 3 steps shifts the
    reordering phase and forces a second capture, a change of decision recording a third."""
    disc = _common_sort_members()[0]
    with B.Discharge(disc) as g, B.Discharge(disc) as e:
        g.set_graph(10)
        replays = 0
        for n in (10, 10, 3, 10, 10, 12):
            g.step(n)
            e.step(n)
            replays += n // 10
            g.sync()
            e.sync()
            assert g.graph_launches() == replays
            _same(_state(g), _state(e), n)
        B.pic_set_record_decisions(g.h, True)
        B.pic_set_record_decisions(e.h, True)
        g.step(10)
        e.step(10)
        assert g.graph_launches() == replays + 1
        _same(_state(g), _state(e), "recording")
        log(f"single-discharge graph replays checked: {replays + 1}")
