"""Write tests/golden/argon_small_ensemble.json: window moments of the FP64 oracle for the
small argon-like discharge (2 cm, 128 cells, 100 V, 20 Pa, 2e4 + 2e4 particles,
dt = T_rf/400), seeds 0..7, averaged over RF cycles 10..20 after a cold start.

Calls only oracle/ and workloads/.  Run:  python tests/golden/make_ensemble.py
"""
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

SEEDS = list(range(8))
CYCLES_SKIP, CYCLES_TOTAL = 10, 20
KEYS = ("n_e", "n_i", "mean_energy_e", "flux_i", "phi")


def run(seed):
    os.environ["OMP_NUM_THREADS"] = "1"
    import numpy as np

    import workloads as W
    from oracle import Oracle
    disc = W.small_argon(seed=seed)
    spp = disc.steps_per_period
    o = Oracle(disc)
    t0 = time.time()
    for _ in range(CYCLES_SKIP * spp):
        o.step()
    o.reset_moments()
    for _ in range((CYCLES_TOTAL - CYCLES_SKIP) * spp):
        o.step()
    m = o.moments()
    out = {k: [float(v) if np.isfinite(v) else None for v in m[k]] for k in KEYS}
    out.update(seed=seed, J0=float(m["J0"]), flux_i_powered=float(m["flux_i_powered"]),
               n_samples=int(m["n_samples"]), alive=[len(o.sp[0].x), len(o.sp[1].x)],
               next_id=[o.sp[0].next_id, o.sp[1].next_id], seconds=time.time() - t0)
    return out


def main():
    with Pool(min(8, len(SEEDS))) as p:
        res = p.map(run, SEEDS)
    import workloads as W
    disc = W.small_argon()
    doc = {"workload": disc.name, "seeds": SEEDS, "cycles": [CYCLES_SKIP, CYCLES_TOTAL],
           "steps_per_period": disc.steps_per_period, "runs": res}
    with open(os.path.join(HERE, "argon_small_ensemble.json"), "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    for r in res:
        print(r["seed"], r["alive"], r["next_id"], f"J0={r['J0']:.3f}", f"{r['seconds']:.0f}s")


if __name__ == "__main__":
    main()
