"""Surrogate warm start: predict the periodic state of a discharge from its parameters and
start the PIC/MCC run from it instead of from a uniform plasma.

Basis in the paper: the periodic state does not depend on the initial density and mean
energy, and reaching it from a uniform start takes ~1000 (low pressure) to ~4000 (high
pressure) RF periods (Sec. 3, on initial values).  A prediction of that state only
shortens the relaxation; the PIC/MCC run still decides the result, and the cold start
remains the reference for the prediction's error.

Pieces (host logic; every particle, field and network operation runs in the HIP library):

* ``SteadyState``: the criterion applied once per RF period (a reading; the paper states
  none).  Period c is steady when, over the last W = 20 periods, (i) the ions created
  (ionisations) and the ions absorbed at both electrodes agree within 3 %, and (ii) the
  W-period mean profiles of n_e, n_i, <eps_e>, phi and Gamma_i differ from those of the W
  periods before by less than 1 % (root-mean-square difference over the grid, relative
  to the larger profile's maximum magnitude), for every quantity.
* ``run``: a batch of discharges (``Batch``: one launch per step for all, one captured
  HIP graph per RF period), cold or warm-loaded, advanced period by period until every
  discharge has been steady for W more periods (its final window) or a period limit.
* ``encode`` / ``decode``: network inputs (p, V0, d, gas id) scaled to [-1, 1]; outputs
  are 5 profiles x 128 points: log10 n_e, log10 n_i (floor 1e12 m^-3), <eps_e> [eV],
  phi / V0 and Gamma_i / 1e19 m^-2 s^-1, each standardised per point over the training
  set.
* ``train``: Adam on the GPU network (``Mlp``, BF16 matrix cores).
* ``evaluate``: held-out parameter draws, each advanced cold and warm in one batch:
  periods to steady state both ways and the warm run's final profiles against the cold
  run's (3 % accuracy).

Command line (run from the repository root on a GPU):
  python -m paper_1608_04601_amd.warmstart generate --n 128 --periods 1200 --out <data.npz>
  python -m paper_1608_04601_amd.warmstart train --data <data.npz> --out <weights.npz>
  python -m paper_1608_04601_amd.warmstart evaluate --weights <weights.npz> --n 16 --periods 1500
"""
import argparse
import json
import os
import sys
import time

import numpy as np

from . import binding as B

DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")
DATA_PATH = os.path.join(DATA_DIR, "steady_states_seed1.npz")
# training draws: seeds 1 and 3 to 9 (seed 2 is held out)
DATA_PATHS = tuple(os.path.join(DATA_DIR, f"steady_states_seed{s}.npz") for s in (1, 3, 4, 5, 6, 7, 8, 9))
N_POINTS = 128
QUANTITIES = ("n_e", "n_i", "mean_energy_e", "phi", "flux_i")
WIDTH, DEPTH = 256, 3
DENSITY_FLOOR = 1e12
FLUX_SCALE = 1e19


def load_data(paths=None):
    """The stored steady states of every training draw that is present, concatenated:
    params, profiles, steady_at, periods, extinct, alive."""
    paths = [p for p in (DATA_PATHS if paths is None else paths) if os.path.exists(p)]
    if not paths:
        raise FileNotFoundError("no stored steady states")
    parts = [np.load(p) for p in paths]
    return {k: np.concatenate([d[k] for d in parts]) for k in parts[0].files}


def training_mask(data):
    """The draws whose stored profiles are periodic steady states: not extinct, and the
    steady-state criterion met (draws still drifting at the period limit are left out)."""
    return ~data["extinct"] & (data["steady_at"] >= 0)


# ------------------------------------------------------------------ steady state
def profile_change(a, b):
    """Per quantity: RMS of a - b over the grid, relative to the larger max |.| of a, b."""
    out = []
    for q in range(a.shape[0]):
        scale = max(np.abs(a[q]).max(), np.abs(b[q]).max(), 1e-300)
        out.append(float(np.sqrt(np.mean((a[q] - b[q]) ** 2)) / scale))
    return np.array(out)


class SteadyState:
    """Periodic-steady-state criterion of one discharge, fed once per RF period."""

    def __init__(self, window=20, balance=0.03, change=0.01):
        self.W, self.balance, self.change = window, balance, change
        self.profiles, self.created, self.absorbed = [], [], []
        self.steady_at = None   # periods completed when the criterion first held

    @property
    def periods(self):
        return len(self.profiles)

    def add(self, prof, created, absorbed):
        self.profiles.append(np.asarray(prof, dtype=np.float64))
        self.created.append(float(created))
        self.absorbed.append(float(absorbed))
        if self.steady_at is None and self.test():
            self.steady_at = self.periods
        return self.steady_at is not None

    def window_mean(self, end=None):
        end = self.periods if end is None else end
        return np.mean(self.profiles[end - self.W:end], axis=0)

    def test(self):
        W, n = self.W, self.periods
        if n < 2 * W:
            return False
        cr, ab = sum(self.created[n - W:]), sum(self.absorbed[n - W:])
        if ab <= 0.0 or abs(cr - ab) > self.balance * ab:
            return False
        return bool(np.all(profile_change(self.window_mean(n), self.window_mean(n - W)) < self.change))

    def done(self):
        """Steady, and W more periods recorded for the final window."""
        return self.steady_at is not None and self.periods >= self.steady_at + self.W


def resample(z_nodes, values, gap, n_points=N_POINTS):
    return np.interp(np.linspace(0.0, gap, n_points), z_nodes, values)


def period_profiles(view, disc):
    """The window means since the last call (one RF period), on N_POINTS points."""
    m = view.moments(reset=True)
    z = np.linspace(0.0, disc.gap_m, disc.n_cells + 1)
    prof = []
    for q in QUANTITIES:
        v = np.nan_to_num(m[q], nan=0.0)   # mean energy is undefined where n_e = 0
        prof.append(resample(z, v, disc.gap_m))
    return np.array(prof)


def run(discs, max_periods, warm=None, stream=None, log=None, max_seconds=None, continue_to=None):
    """Advance the discharges (one batch) period by period; warm[k] (or None) holds the
    profiles (n_e, n_i, mean_energy_e, flux_i) that discharge k starts from.  Stops when
    every discharge is steady, after max_periods, or once max_seconds have passed.  With
    continue_to, every discharge keeps running (and recording its profiles) until that many
    periods even after it became steady, so that the final windows show where the
    discharges go after the criterion first held.  Returns one dict per discharge:
    steady_at, periods, final (the last W-period mean profiles), drift (the criterion's
    profile change between the last two windows), alive (electrons and ions at the end),
    extinct."""
    spp = {int(round(1.0 / (d.rf_frequency_Hz * d.dt_s))) for d in discs}
    if len(spp) != 1:
        raise ValueError("all discharges of a run need the same steps per RF period")
    spp = spp.pop()
    bt = B.Batch(discs, stream=stream)
    try:
        if warm is not None:
            for k, w in enumerate(warm):
                if w is not None:
                    B.pic_load_profiles(bt[k].h, w["n_e"], w["n_i"], w["mean_energy_e"], w["flux_i"])
        bt.rebalance()   # a warm load changes the particle counts
        bt.set_graph(spp)
        det = [SteadyState() for _ in discs]
        prev = [(bt[k].counters()["births_total"], int(bt[k].counters()["absorbed_total"][1].sum()))
                for k in range(len(discs))]
        for k in range(len(discs)):
            bt[k].moments(reset=True)
        t0 = t_log = time.time()
        for c in range(max_periods):
            if c % 50 == 49:
                bt.rebalance()   # the counts drift while the discharges relax
            bt.step(spp)
            bt.sync()
            for k, d in enumerate(discs):
                if det[k].done() and continue_to is None:
                    continue
                cnt = bt[k].counters()
                born, lost = cnt["births_total"], int(cnt["absorbed_total"][1].sum())
                det[k].add(period_profiles(bt[k], d), born - prev[k][0], lost - prev[k][1])
                prev[k] = (born, lost)
            if log and ((c + 1) % 100 == 0 or time.time() - t_log > 60.0):   # at least once a minute
                t_log = time.time()
                n_done = sum(x.done() for x in det)
                log(f"  period {c + 1}: {n_done}/{len(discs)} steady, {t_log - t0:.0f} s")
            if all(x.done() for x in det) and (continue_to is None or c + 1 >= continue_to):
                break
            if max_seconds is not None and time.time() - t0 > max_seconds:
                if log:
                    log(f"  stopped after {c + 1} periods at the {max_seconds:.0f} s limit")
                break
        out = []
        for k, d in enumerate(discs):
            cnt = bt[k].counters()
            n, W = det[k].periods, det[k].W
            drift = (profile_change(det[k].window_mean(n), det[k].window_mean(n - W)).tolist()
                     if n >= 2 * W else None)   # change between the last two windows
            out.append(dict(steady_at=det[k].steady_at, periods=n, final=det[k].window_mean(), drift=drift,
                            alive=tuple(cnt["n_alive"]), extinct=cnt["n_alive"][0] < 100))
        return out
    finally:
        bt.close()


# ------------------------------------------------------------------ network I/O
def encode_inputs(params):
    p = np.asarray(params, dtype=np.float64)
    return np.stack([(p[:, 0] - 45.0) / 35.0, (p[:, 1] - 250.0) / 150.0, (p[:, 2] - 0.025) / 0.005,
                     2.0 * p[:, 3] - 1.0], axis=1).astype(np.float32)


def to_targets(params, profiles):
    """profiles [K x 5 x N_POINTS] -> untransformed network targets [K x 5 N_POINTS]."""
    pr = np.asarray(profiles, dtype=np.float64)
    v0 = np.asarray(params, dtype=np.float64)[:, 1][:, None]
    t = [np.log10(np.maximum(pr[:, 0], DENSITY_FLOOR)), np.log10(np.maximum(pr[:, 1], DENSITY_FLOOR)), pr[:, 2],
         pr[:, 3] / v0, pr[:, 4] / FLUX_SCALE]
    return np.concatenate(t, axis=1)


def from_targets(params, t):
    t = np.asarray(t, dtype=np.float64).reshape(len(t), 5, N_POINTS)
    v0 = np.asarray(params, dtype=np.float64)[:, 1][:, None]
    return np.stack([10.0 ** t[:, 0], 10.0 ** t[:, 1], np.maximum(t[:, 2], 0.0), t[:, 3] * v0,
                     t[:, 4] * FLUX_SCALE], axis=1)


def train(params, profiles, steps=4000, lr=1e-3, seed=0, stream=None, log=None):
    """Fit the network to (params -> profiles); returns (Mlp, normalisation, final loss)."""
    import torch
    X = encode_inputs(params)
    T = to_targets(params, profiles)
    mu, sd = T.mean(axis=0), np.maximum(T.std(axis=0), 1e-3)
    Tn = ((T - mu) / sd).astype(np.float32)
    net = B.Mlp(4, WIDTH, DEPTH, 5 * N_POINTS, max_batch=len(X), seed=seed, stream=stream)
    xd = torch.from_numpy(X).cuda()
    td = torch.from_numpy(Tn).cuda()
    loss = None
    for it in range(steps):
        rate = lr if it < steps // 2 else (lr * 0.3 if it < 3 * steps // 4 else lr * 0.1)
        want = it == steps - 1 or (log is not None and it % 1000 == 0)
        loss = net.train_step(xd, td, rate, want_loss=want)
        if log and want:
            log(f"  train step {it}: loss {loss:.4e}")
    return net, dict(mu=mu, sd=sd), loss


def predict(net, norm, params):
    """Profiles [K x 5 x N_POINTS] predicted for the parameter rows."""
    import torch
    X = torch.from_numpy(encode_inputs(params)).cuda()
    Y = torch.empty(len(params), 5 * N_POINTS, device="cuda")
    net.forward(X, Y)
    torch.cuda.synchronize()
    return from_targets(params, Y.cpu().numpy() * norm["sd"] + norm["mu"])


def warm_profiles(prof):
    """Loader input from predicted profiles, or None (the discharge then starts cold, the
    plain method) when the prediction is not finite."""
    if not np.all(np.isfinite(prof)):
        return None
    return dict(n_e=prof[0], n_i=prof[1], mean_energy_e=prof[2], flux_i=prof[4])


# ------------------------------------------------------------------ command line
def _log(msg):
    print(msg, flush=True)


def cmd_generate(a):
    import workloads as W
    params = W.surrogate_params(a.n, a.seed)
    discs = [W.surrogate_discharge(params[k], k, seed=a.seed) for k in range(a.n)]
    _log(f"generate: {a.n} discharges, up to {a.periods} periods")
    res = run(discs, a.periods, log=_log)
    np.savez(a.out, params=params, profiles=np.array([r["final"] for r in res]),
             steady_at=np.array([-1 if r["steady_at"] is None else r["steady_at"] for r in res]),
             periods=np.array([r["periods"] for r in res]), extinct=np.array([r["extinct"] for r in res]),
             alive=np.array([r["alive"] for r in res]))
    _log(f"generate: steady {sum(r['steady_at'] is not None for r in res)}/{a.n}, "
         f"extinct {sum(r['extinct'] for r in res)}; wrote {a.out}")


def cmd_train(a):
    data = np.load(a.data)
    keep = training_mask(data)
    _log(f"train: {keep.sum()} steady states (extinct draws and draws not steady at the limit left out)")
    net, norm, loss = train(data["params"][keep], data["profiles"][keep], steps=a.steps, seed=a.seed, log=_log)
    np.savez(a.out, theta=net.get_params(), mu=norm["mu"], sd=norm["sd"], loss=loss,
             shape=np.array([4, WIDTH, DEPTH, 5 * N_POINTS]))
    _log(f"train: final loss {loss:.4e}; wrote {a.out}")


def load_net(path, stream=None):
    w = np.load(path)
    n_in, width, depth, n_out = (int(v) for v in w["shape"])
    net = B.Mlp(n_in, width, depth, n_out, max_batch=1024, stream=stream)
    net.set_params(w["theta"])
    return net, dict(mu=w["mu"], sd=w["sd"])


def evaluate(net, norm, params, seed, max_periods, log=None, index=None):
    """Cold and warm runs of the same held-out discharges in one batch; index[k] (default k)
    is discharge k's position in its draw, which keys its random numbers."""
    import workloads as W
    K = len(params)
    pred = predict(net, norm, params)
    index = list(range(K)) if index is None else list(index)
    discs = [W.surrogate_discharge(params[k], index[k], seed=seed) for k in range(K)]
    warm = [None] * K + [warm_profiles(pred[k]) for k in range(K)]
    res = run(discs + discs, max_periods, warm=warm, log=log)
    rows = []
    for k in range(K):
        cold, hot = res[k], res[K + k]
        rows.append(dict(params=[float(v) for v in params[k]], cold_steady_at=cold["steady_at"],
                         warm_steady_at=hot["steady_at"], extinct=bool(cold["extinct"] or hot["extinct"]),
                         warm_vs_cold=profile_change(hot["final"], cold["final"]).tolist(),
                         prediction_vs_cold=profile_change(pred[k], cold["final"]).tolist(),
                         periods_run=[cold["periods"], hot["periods"]]))
    return rows


def evaluate_discharge(net, norm, disc, gas_id, max_periods, log=None, max_seconds=None, continue_to=None):
    """One discharge of any fidelity, cold and warm in one batch.  The network sees its
    (p, V0, d, gas id); the prediction is resampled onto the loader's points."""
    params = np.array([[disc.pressure_Pa, disc.rf_voltage_V, disc.gap_m, float(gas_id)]])
    pred = predict(net, norm, params)[0]
    res = run([disc, disc], max_periods, warm=[None, warm_profiles(pred)], log=log, max_seconds=max_seconds,
              continue_to=continue_to)
    cold, hot = res
    return dict(params=[float(v) for v in params[0]], cold_steady_at=cold["steady_at"], warm_steady_at=hot["steady_at"],
                extinct=bool(cold["extinct"] or hot["extinct"]), warm_vs_cold=profile_change(hot["final"], cold["final"]).tolist(),
                prediction_vs_cold=profile_change(pred, cold["final"]).tolist(), alive_cold=cold["alive"],
                alive_warm=hot["alive"], periods_run=[cold["periods"], hot["periods"]],
                drift_cold=cold["drift"], drift_warm=hot["drift"])


def summarize(rows, max_periods):
    ok = [r for r in rows if not r["extinct"]]
    both = [r for r in ok if r["cold_steady_at"] is not None and r["warm_steady_at"] is not None]
    # a run that is not steady counts with the periods it ran (a lower bound: the period
    # limit, or fewer when a time limit stopped it)
    ran = [r.get("periods_run", (max_periods, max_periods)) for r in ok]
    cold = [r["cold_steady_at"] if r["cold_steady_at"] is not None else n[0] for r, n in zip(ok, ran)]
    warm = [r["warm_steady_at"] if r["warm_steady_at"] is not None else n[1] for r, n in zip(ok, ran)]
    acc = [max(r["warm_vs_cold"]) for r in both]
    return dict(discharges=len(rows), extinct=len(rows) - len(ok), steady_both=len(both),
                cold_periods_mean=float(np.mean(cold)) if cold else None,
                warm_periods_mean=float(np.mean(warm)) if warm else None,
                cold_not_steady=sum(r["cold_steady_at"] is None for r in ok),
                warm_not_steady=sum(r["warm_steady_at"] is None for r in ok),
                warm_faster=sum(r["warm_steady_at"] is not None and w < c for r, w, c in zip(ok, warm, cold)),
                warm_vs_cold_max=float(max(acc)) if acc else None,
                warm_vs_cold_median=float(np.median(acc)) if acc else None,
                within_3pct=sum(a <= 0.03 for a in acc),
                prediction_vs_cold_median=float(np.median([max(r["prediction_vs_cold"]) for r in ok])) if ok else None)


def cmd_evaluate(a):
    import workloads as W
    net, norm = load_net(a.weights)
    params = W.surrogate_params(a.n, a.seed)
    _log(f"evaluate: {a.n} held-out discharges, cold and warm, up to {a.periods} periods")
    rows = evaluate(net, norm, params, a.seed, a.periods, log=_log)
    out = dict(summary=summarize(rows, a.periods), rows=rows)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(out, f, indent=1)
    _log(json.dumps(out["summary"]))


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1608_04601_amd.warmstart")
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--n", type=int, default=128)
    g.add_argument("--seed", type=int, default=1)
    g.add_argument("--periods", type=int, default=1200)
    g.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--data", required=True)
    t.add_argument("--steps", type=int, default=4000)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--out", required=True)
    e = sub.add_parser("evaluate")
    e.add_argument("--weights", required=True)
    e.add_argument("--n", type=int, default=16)
    e.add_argument("--seed", type=int, default=2)
    e.add_argument("--periods", type=int, default=1500)
    e.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    {"generate": cmd_generate, "train": cmd_train, "evaluate": cmd_evaluate}[a.cmd](a)


if __name__ == "__main__":
    sys.exit(main())
