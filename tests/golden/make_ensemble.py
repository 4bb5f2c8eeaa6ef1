"""Write the statistical-parity golden files from the FP64 oracle: window moments averaged
over RF cycles after a cold start, seeds 0..7, for
* argon_small_ensemble.json: the small argon-like discharge (2 cm, 128 cells, 100 V, 20 Pa,
  2e4 + 2e4 particles, dt = T_rf/400), cycles 10..20;
* helium_small_ensemble.json: the small helium-like discharge (2.5 cm, 128 cells, 200 V,
  40 Pa, 2e4 + 2e4 particles, dt = T_rf/800), cycles 10..20;
* argon_4096c_ensemble.json: the large argon-like discharge's geometry (3 cm, 4096 cells,
  300 V, 80 Pa, dt = T_rf/4000) with 5e4 + 5e4 particles at the start, cycles 4..8.

Calls only oracle/ and workloads/.
Run:  python tests/golden/make_ensemble.py [argon|helium|large]
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
KEYS = ("n_e", "n_i", "mean_energy_e", "flux_i", "phi")

# workload, its arguments, output file, (cycles skipped, cycles total)
CASES = {"argon": ("small_argon", {}, "argon_small_ensemble.json", (10, 20)),
         "helium": ("small_helium", {}, "helium_small_ensemble.json", (10, 20)),
         "large": ("large_argon", {"n_super": 50_000}, "argon_4096c_ensemble.json", (4, 8))}


def run(args):
    case, seed = args
    os.environ["OMP_NUM_THREADS"] = "1"
    import numpy as np

    import workloads as W
    from oracle import Oracle
    name, kw, _, (skip, total) = CASES[case]
    disc = getattr(W, name)(seed=seed, **kw)
    spp = disc.steps_per_period
    o = Oracle(disc)
    t0 = time.time()
    for _ in range(skip * spp):
        o.step()
    o.reset_moments()
    for _ in range((total - skip) * spp):
        o.step()
    m = o.moments()
    out = {k: [float(v) if np.isfinite(v) else None for v in m[k]] for k in KEYS}
    out.update(seed=seed, J0=float(m["J0"]), flux_i_powered=float(m["flux_i_powered"]),
               n_samples=int(m["n_samples"]), alive=[len(o.sp[0].x), len(o.sp[1].x)],
               next_id=[o.sp[0].next_id, o.sp[1].next_id], seconds=time.time() - t0)
    return out


def main():
    case = sys.argv[1] if len(sys.argv) > 1 else "argon"
    with Pool(min(8, len(SEEDS))) as p:
        res = p.map(run, [(case, s) for s in SEEDS])
    import workloads as W
    name, kw, out, (skip, total) = CASES[case]
    disc = getattr(W, name)(**kw)
    doc = {"workload": disc.name, "seeds": SEEDS, "cycles": [skip, total],
           "steps_per_period": disc.steps_per_period, "runs": res}
    with open(os.path.join(HERE, out), "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    for r in res:
        print(r["seed"], r["alive"], r["next_id"], f"J0={r['J0']:.3f}", f"{r['seconds']:.0f}s")


if __name__ == "__main__":
    main()
