"""Parity at full size, in the launch configuration bench.py times (automatic workgroup
count, no decision recording): the production discharge (1e6 particles per species, 512
cells) and the large one (2.5e7 per species, 4096 cells).  From the GPU's own state at step
100 (after reorderings: every 20 and every 50 steps respectively), the oracle takes the
whole state through one step.

* The field of that state (deposit and Poisson) agrees within 1e-5 of its maximum.
* After the step: fields within 1e-5; every particle's position within 1e-5 d (positions
  of step n + 1 do not depend on that step's collisions); velocities within 1e-5
  max(|v|, v_th) for all but the particles whose collision choice fell in the margin band
  of the FP32 test (at most 1e-4 of them); alive counts within that many.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import REL_FIELD, REL_V, REL_X, gpu_species, log, oracle_input, vth
from oracle import Oracle
from paper_1608_04601_amd import binding as B

pytestmark = pytest.mark.gpu

CASES = {"production_helium": W.production_helium, "large_argon": W.large_argon}


@pytest.mark.parametrize("name", list(CASES))
def test_full_size_single_step(name):
    disc = CASES[name]()
    log(f"full-size parity: {name} N={disc.n_super} cells={disc.n_cells}")
    with B.Discharge(disc) as d:
        # the launch the benchmark times: the dynamic work distribution at 4096 cells
        assert d.launch_shape()[2] == (name == "large_argon")
        d.step(100)
        c0 = d.counters()
        o = Oracle(disc, load=False)
        o.set_state(c0["step"], oracle_input(d, c0))
        f0 = d.fields()
        assert np.max(np.abs(f0["E"] - o.E)) <= REL_FIELD * np.abs(o.E).max()
        d.step(1)
        o.step()
        f = d.fields()
        assert np.max(np.abs(f["E"] - o.E)) <= REL_FIELD * np.abs(o.E).max()
        assert np.max(np.abs(f["phi"] - o.phi)) <= REL_FIELD * max(np.abs(o.phi).max(), disc.rf_voltage_V)
        c1 = d.counters()
        for s in (0, 1):
            g = gpu_species(d, s)
            S = o.state(s)
            common, ig, io = np.intersect1d(g["id"].astype(np.int64), S["id"].astype(np.int64),
                                            assume_unique=True, return_indices=True)
            n = len(S["id"])
            allowed = max(4, int(1e-4 * n))
            assert len(common) >= n - allowed and abs(c1["n_alive"][s] - n) <= allowed
            dx = np.abs(g["x"][ig] - S["x"][io])
            assert dx.max() <= REL_X * disc.gap_m, (s, dx.max())
            vo = np.stack([S["vx"][io], S["vy"][io], S["vz"][io]], axis=1)
            scale = np.maximum(np.max(np.abs(vo), axis=1), vth(o, s))
            dv = np.max(np.abs(np.stack([g["vx"][ig], g["vy"][ig], g["vz"][ig]], axis=1) - vo), axis=1)
            bad = int(np.sum(dv > REL_V * scale))
            log(f"  species {s}: {n} particles, {len(common)} common ids, velocity outliers {bad}")
            assert bad <= allowed
