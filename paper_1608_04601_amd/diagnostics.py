"""Drivers for the results-section diagnostics (pic_diag_*, pic_electrode_fluxes).

* ``phase_resolved``: profiles at a fixed phase t f of the RF period, averaged over periods
  (the paper compares its models at t f = 0.25, when the powered electrode is at +V0):
  E, n_e, U_e, the heating rate -e0 E Gamma_e, the ionisation rate S, Gamma_e, Q_e and the
  density of fast electrons (U > e0 V0 / 4).
* ``time_averaged``: the same quantities and the isotropic distribution f0(U)/n_e averaged
  over whole periods, sampled every ``every`` steps.
* ``electrode_fluxes``: Gamma_e(t) and Gamma_i(t) at the powered electrode over the last
  period.

Command line (on a GPU, from the repository root): a discharge of ``workloads`` is relaxed
for some periods, then sampled, and the result written as JSON:
  python -m paper_1608_04601_amd.diagnostics --workload small --relax 20 --periods 10 --out <file.json>
"""
import argparse
import json
import sys

import numpy as np

from . import binding as B


def _steps_per_period(disc):
    return int(round(1.0 / (disc.rf_frequency_Hz * disc.dt_s)))


def phase_resolved(d, disc, periods, phase=0.25, n_bins=200, u_max_eV=100.0):
    """Step the discharge handle d whole periods, sampling once per period at t f = phase
    (the discharge must stand at the start of a period)."""
    spp = _steps_per_period(disc)
    k = int(round(phase * spp)) % spp
    B.pic_diag_config(d.h, n_bins, u_max_eV)
    for _ in range(periods):
        d.step(k)
        B.pic_diag_sample(d.h)
        d.step(spp - k)
    return B.pic_diag_read(d.h, disc.n_cells + 1, n_bins, reset=True)


def time_averaged(d, disc, periods, every=50, n_bins=200, u_max_eV=100.0):
    """Sample every `every` steps over whole periods (every must divide the period)."""
    spp = _steps_per_period(disc)
    if spp % every:
        raise ValueError("every must divide the steps per RF period")
    B.pic_diag_config(d.h, n_bins, u_max_eV)
    for _ in range(periods * spp // every):
        d.step(every)
        B.pic_diag_sample(d.h)
    return B.pic_diag_read(d.h, disc.n_cells + 1, n_bins, reset=True)


def electrode_fluxes(d, disc):
    return B.pic_electrode_fluxes(d.h, _steps_per_period(disc))


def _jsonable(r):
    return {k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in r.items()}


def main(argv=None):
    import workloads as W
    ap = argparse.ArgumentParser(prog="python -m paper_1608_04601_amd.diagnostics")
    ap.add_argument("--workload", default="small", choices=("small", "production"))
    ap.add_argument("--relax", type=int, default=20, help="RF periods before sampling")
    ap.add_argument("--periods", type=int, default=10)
    ap.add_argument("--phase", type=float, default=0.25)
    ap.add_argument("--every", type=int, default=50)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    disc = W.small_argon() if a.workload == "small" else W.production_helium()
    spp = _steps_per_period(disc)
    with B.Discharge(disc) as d:
        d.step(a.relax * spp)
        ph = phase_resolved(d, disc, a.periods, a.phase)
        ta = time_averaged(d, disc, a.periods, a.every)
        ge, gi = electrode_fluxes(d, disc)
    out = dict(workload=disc.name, phase=a.phase, phase_resolved=_jsonable(ph), time_averaged=_jsonable(ta),
               gamma_e_powered=ge.tolist(), gamma_i_powered=gi.tolist())
    with open(a.out, "w") as f:
        json.dump(out, f)
    print(f"wrote {a.out}: {ph['n_samples']} phase samples, {ta['n_samples']} time samples", flush=True)


if __name__ == "__main__":
    sys.exit(main())
