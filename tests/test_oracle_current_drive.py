"""Pin of the oracle's current-driven RF amplitude (Sec. 2, Eq. "adaptivevoltage") on a
vacuum gap, where the closed form is known: with no charge the electrode field is
V0 sin(w t) / d, the current is the displacement current eps0 dE/dt, and its discrete
amplitude over a whole period of N steps is
    J_amp(V0) = eps0 V0 2 sin(w dt / 2) cos(pi / N) / (d dt),
linear in V0; one adaptation therefore gives V0 = J0 / (J_amp(V0) / V0) and the next
period's amplitude equals J0."""
import numpy as np

import workloads as W
from oracle import Oracle
from oracle.constants import EPS0


def _vacuum(disc):
    o = Oracle(disc, load=False)
    empty = dict(x=np.zeros(0), vx=np.zeros(0), vy=np.zeros(0), vz=np.zeros(0), id=np.zeros(0, np.uint64),
                 next_id=0)
    o.set_state(0, [empty, dict(empty)])
    o.reset_moments()
    return o


def test_vacuum_gap_reaches_the_target_current_in_one_period():
    J0 = 12.5
    disc = W.small_argon(seed=0, n_super=100).replace(j0_target_A_m2=J0)
    N = disc.steps_per_period
    w = 2.0 * np.pi * disc.rf_frequency_Hz
    per_volt = EPS0 * 2.0 * np.sin(w * disc.dt_s / 2.0) * np.cos(np.pi / N) / (disc.gap_m * disc.dt_s)
    o = _vacuum(disc)
    amps = []
    for period in range(3):
        jmax = 0.0
        for _ in range(N):
            o.step()
            jmax = max(jmax, abs(o.J))
        amps.append(jmax)
        if period == 0:
            np.testing.assert_allclose(jmax, disc.rf_voltage_V * per_volt, rtol=1e-9)
            np.testing.assert_allclose(o.V0, J0 / per_volt, rtol=1e-9)
    np.testing.assert_allclose(amps[1:], J0, rtol=1e-9)


def test_without_a_target_the_amplitude_is_prescribed():
    disc = W.small_argon(seed=0, n_super=100)
    o = _vacuum(disc)
    for _ in range(2 * disc.steps_per_period):
        o.step()
    assert o.V0 == disc.rf_voltage_V
