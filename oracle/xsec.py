"""Cross-section lookup and the null-collision bound (Sec. 2.5 null-collision method;
Sec. 4.1 and Table "tab:reactions" for the processes, the ion energy floor and the
energy frames).

Readings (the paper gives the data only as figures):
  * a table holds sigma at eps_k = k * de for k = 0..K-1;
  * sigma(eps) = 0 below the threshold, the last value at or above the last point,
    otherwise linear interpolation, eps first clamped up to the table's floor;
  * a LAB table is read at 1/2 m_s g^2 / e0, a CM table at 1/2 mu g^2 / e0, with g the
    speed relative to the gas atom and mu = m_s M / (m_s + M);
  * the collision frequency of a particle is n_gas * sum_j sigma_j * g;
  * nu_max is the supremum of that frequency over the table range (the largest last
    table point, in lab energy), found exactly segment by segment;
  * the candidate threshold is T = round-half-even(2^24 * (1 - exp(-nu_max dt))).
"""
import numpy as np

from .constants import E0


def sigma_lookup(proc, eps):
    """sigma_j(eps) [m^2] for frame energies eps [eV] (array)."""
    eps = np.asarray(eps, dtype=np.float64)
    tab = np.asarray(proc.sigma_m2, dtype=np.float64)
    K = tab.shape[0]
    e = np.maximum(eps, proc.emin_eV)
    t = e / proc.de_eV
    k = np.floor(t)
    kk = np.clip(k, 0, K - 2).astype(np.int64)
    frac = t - kk
    s = tab[kk] + (tab[kk + 1] - tab[kk]) * frac
    s = np.where(k >= K - 1, tab[K - 1], s)
    return np.where(eps < proc.threshold_eV, 0.0, s)


def frame_factor(proc, m_s, M):
    """Frame energy per lab energy: 1 for LAB, mu/m_s = M/(m_s+M) for CM."""
    return 1.0 if proc.frame == 0 else M / (m_s + M)


def energy_factor(proc, m_s, M):
    """Frame energy [eV] per g^2 [m^2/s^2]."""
    m_frame = m_s if proc.frame == 0 else m_s * M / (m_s + M)
    return 0.5 * m_frame / E0


def nu_max(procs, m_s, M, n_gas):
    """sup over lab energies in [0, top] of n_gas * sum_j sigma_j(c_j eps) * sqrt(2 e0 eps / m_s)."""
    if not procs:
        return 0.0
    c = [frame_factor(p, m_s, M) for p in procs]
    top = max((len(p.sigma_m2) - 1) * p.de_eV / cj for p, cj in zip(procs, c))
    bps = [np.array([0.0, top])]
    for p, cj in zip(procs, c):
        K = len(p.sigma_m2)
        bps.append(np.arange(K, dtype=np.float64) * p.de_eV / cj)
        bps.append(np.array([p.threshold_eV / cj, p.emin_eV / cj]))
    b = np.unique(np.concatenate(bps))
    b = b[(b >= 0.0) & (b <= top)]
    lo, hi = b[:-1], b[1:]
    keep = hi > lo
    lo, hi = lo[keep], hi[keep]

    def ssum(eps):
        return sum(sigma_lookup(p, cj * eps) for p, cj in zip(procs, c))

    # sum of sigma is linear on each open segment: recover it from two interior points
    m1 = lo + (hi - lo) / 3.0
    m2 = lo + 2.0 * (hi - lo) / 3.0
    s1, s2 = ssum(m1), ssum(m2)
    beta = (s2 - s1) / (m2 - m1)
    alpha = s1 - beta * m1
    cands = [lo, hi]
    with np.errstate(divide="ignore", invalid="ignore"):
        st = np.where(beta < 0.0, -alpha / (3.0 * beta), -1.0)
    inside = (st > lo) & (st < hi)
    cands.append(np.where(inside, st, lo))
    best = 0.0
    for e in cands:
        sig = np.maximum(alpha + beta * e, 0.0)
        f = sig * np.sqrt(2.0 * E0 * e / m_s)
        best = max(best, float(f.max()))
    return n_gas * best


def candidate_threshold(numax, dt):
    """T = round-half-even(2^24 * (1 - exp(-nu_max dt))); a particle is a candidate iff (w0 >> 8) < T."""
    p = -np.expm1(-numax * dt)
    return int(round(p * 2.0 ** 24)), p
