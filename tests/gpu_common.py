"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import sys

import numpy as np

from oracle import Oracle  # noqa: F401  (tests only)

# Tolerances (single step): the GPU keeps particles in FP32, the oracle in FP64.
REL_X = 1e-5        # |dx| <= REL_X * d
REL_V = 1e-5        # |dv| <= REL_V * max(|v|, v_th)
REL_FIELD = 1e-5    # max|dE| <= REL_FIELD * max|E|; max|dphi| <= REL_FIELD * max(|phi|, V0)
MARGIN = 1e-5       # process choices may differ only where |R - c_j| < MARGIN * nu_max


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_species(d, s):
    p = d.particles(s)
    o = np.argsort(p["id"], kind="stable")
    return {k: v[o] for k, v in p.items()}


def oracle_input(d, counters):
    st = []
    for s in (0, 1):
        p = gpu_species(d, s)
        st.append(dict(x=p["x"].astype(np.float64), vx=p["vx"].astype(np.float64), vy=p["vy"].astype(np.float64),
                       vz=p["vz"].astype(np.float64), id=p["id"].astype(np.uint64), next_id=counters["next_id"][s]))
    return st


def vth(o, s):
    from oracle.constants import E0
    T = (o.cfg.te_init_eV, o.cfg.ti_init_eV)[s]
    return np.sqrt(E0 * max(T, 1e-3) / o.d.m[s])
