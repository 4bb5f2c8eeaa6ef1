"""Current-driven operation (Sec. 2, Eq. "adaptivevoltage") on the GPU: V0 <- V0 J0 / J_calc
at the end of every whole RF period.

* Vacuum gap (no particles): the closed form of the discrete displacement-current
  amplitude, J_amp = eps0 V0 2 sin(w dt / 2) cos(pi / N) / (d dt), fixes V0 after one
  adaptation, and every later period's amplitude equals J0.
* Plasma: the amplitude after a period equals V0 J0 / J_calc with J_calc the GPU's own
  period maximum (pic_moments J0 of a one-period window), and one step from the GPU's state
  at the adapted V0 matches the oracle given that V0.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import REL_FIELD, oracle_input
from oracle import Oracle
from oracle.constants import EPS0
from paper_1608_04601_amd import binding as B

pytestmark = pytest.mark.gpu


def test_vacuum_gap_closed_form():
    J0 = 12.5
    disc = W.small_argon(seed=0, n_super=100).replace(j0_target_A_m2=J0)
    N = disc.steps_per_period
    w = 2.0 * np.pi * disc.rf_frequency_Hz
    per_volt = EPS0 * 2.0 * np.sin(w * disc.dt_s / 2.0) * np.cos(np.pi / N) / (disc.gap_m * disc.dt_s)
    nn = disc.n_cells + 1
    empty = np.zeros(0)
    with B.Discharge(disc) as d:
        for s in (0, 1):
            B.pic_set_particles(d.h, s, empty, empty, empty, empty, np.zeros(0, np.uint32), 0, 0)
        B.pic_moments(d.h, nn, reset=True)
        d.step(N)
        m1 = B.pic_moments(d.h, nn, reset=True)
        v1 = d.counters()["V0"]
        np.testing.assert_allclose(m1["J0"], disc.rf_voltage_V * per_volt, rtol=1e-9)
        np.testing.assert_allclose(v1, J0 / per_volt, rtol=1e-9)
        d.step(2 * N)
        m2 = B.pic_moments(d.h, nn, reset=True)
        np.testing.assert_allclose(m2["J0"], J0, rtol=1e-9)
        assert d.counters()["n_alive"] == (0, 0)


def test_plasma_adaptation_and_single_step_parity():
    J0 = 4.0
    disc = W.small_argon(seed=5).replace(j0_target_A_m2=J0)
    N = disc.steps_per_period
    nn = disc.n_cells + 1
    with B.Discharge(disc) as d:
        B.pic_moments(d.h, nn, reset=True)
        d.step(N)
        m = B.pic_moments(d.h, nn, reset=True)
        c = d.counters()
        np.testing.assert_allclose(c["V0"], disc.rf_voltage_V * J0 / m["J0"], rtol=1e-12)
        d.step(7)
        c0 = d.counters()
        o = Oracle(disc, load=False)
        o.V0 = c0["V0"]
        o.set_state(c0["step"], oracle_input(d, c0))
        d.step(1)
        o.step()
        f = d.fields()
        assert np.max(np.abs(f["E"] - o.E)) <= REL_FIELD * np.abs(o.E).max()
        assert np.max(np.abs(f["phi"] - o.phi)) <= REL_FIELD * max(np.abs(o.phi).max(), abs(o.V0))
