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


def compare_decisions(o, s, decisions, next_id_before):
    """Candidates identical; process choices identical outside the margin band.  Returns the
    GPU's choice per candidate id and the ids whose choice legitimately differs."""
    rec = o.last[f"mcc{s}"]
    did, dcode = decisions
    old = did.astype(np.int64) < next_id_before
    did, dcode = did[old].astype(np.int64), dcode[old]
    cand_gpu = np.sort(did[dcode >= 1])
    order = np.argsort(rec["candidates"].astype(np.int64), kind="stable")
    cand_orc = rec["candidates"].astype(np.int64)[order]
    assert np.array_equal(cand_gpu, cand_orc), (s, len(cand_gpu), len(cand_orc))
    gmap = dict(zip(did.tolist(), dcode.tolist()))
    g_sel = np.array([gmap[i] - 2 if gmap[i] >= 2 else -1 for i in cand_orc.tolist()], dtype=np.int64)
    o_sel = rec["selected"][order]
    differ = g_sel != o_sel
    excused = rec["margin"][order] < MARGIN * o.d.numax[s]
    assert np.all(excused[differ]), (s, int(differ.sum()), int((differ & ~excused).sum()))
    return dict(zip(cand_orc.tolist(), g_sel.tolist())), set(cand_orc[differ].tolist())


def compare_species(o, s, g_after, unsure, skip_ids_from, disc):
    """Per-id state after one step; ids in `unsure` and ids >= skip_ids_from are skipped."""
    S = o.state(s)
    gid = g_after["id"].astype(np.int64)
    oid = S["id"].astype(np.int64)
    gid_c = gid[gid < skip_ids_from]
    oid_c = oid[oid < skip_ids_from]
    # the same particles survive (absorption ties at FP32 resolution excepted)
    only_g = np.setdiff1d(gid_c, oid_c)
    only_o = np.setdiff1d(oid_c, gid_c)
    assert len(only_g) + len(only_o) <= 2, (s, only_g[:5], only_o[:5])
    common, ig, io = np.intersect1d(gid, oid, return_indices=True)
    keep = np.array([(i not in unsure) and i < skip_ids_from for i in common.tolist()], dtype=bool)
    ig, io = ig[keep], io[keep]
    dx = np.abs(g_after["x"][ig] - S["x"][io])
    assert dx.max(initial=0) <= REL_X * disc.gap_m, (s, dx.max())
    vt = vth(o, s)
    for key in ("vx", "vy", "vz"):
        ref = S[key][io]
        dv = np.abs(g_after[key][ig] - ref)
        lim = REL_V * np.maximum(np.abs(ref), vt)
        bad = dv > lim
        assert not bad.any(), (s, key, int(bad.sum()), float((dv / lim).max()))
    return len(ig)
