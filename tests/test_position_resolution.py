"""Resolution of FP32 particle positions on the large grid (3 cm, 4096 cells, dt = T_rf/4000).

The GPU keeps positions in FP32 cell units, t = x/dx, and drifts them as t <- fma(v_x, dt/dx,
t).  Between t = 2048 and the electrode at 4096 the FP32 spacing is 2^-12 = 2.4e-4 cells,
while a thermal argon ion (300 K) moves about 6e-4 cells per step: the drift is rounded to
whole spacings, so an ion's speed between collisions is in effect quantised in steps of
2^-12 dx/dt = 97 m/s.  These tests measure what that does to ion transport (the ion density
and flux profiles follow from the drift and the spread of the ions) against the same ions
with FP64 positions and the same FP32 velocities: the mean displacement (drift, hence the
flux) and its variance (diffusion), over 10^4 steps (2.5 RF periods, about one mean free
time) with charge exchange at the 80 Pa rate of the large argon discharge and a 300 V/m bulk
field.  The velocity arithmetic mirrors the kernel (FP32 half kicks), so only the position
encoding differs between the two runs.
"""
import numpy as np

from oracle.constants import AMU, E0, KB

GAP, CELLS, F_RF = 0.03, 4096, 13.56e6
DT = 1.0 / (F_RF * 4000)
DX = GAP / CELLS
M_AR = 39.948 * AMU
T_GAS = 300.0
N_GAS = 80.0 / (KB * T_GAS)
SIGMA_CX = 5e-19


def _fma32(a, b, c):
    """FP32 fused multiply-add: the FP32 product is exact in FP64, one rounding to FP32."""
    return (a.astype(np.float64) * np.float64(b) + c.astype(np.float64)).astype(np.float32)


def _transport(n=20_000, steps=10_000, e_field=300.0, seed=0):
    rng = np.random.default_rng(seed)
    vth = np.sqrt(KB * T_GAS / M_AR)
    t32 = rng.uniform(2200.0, 3800.0, n).astype(np.float32)   # cell units, the coarsest FP32 band
    x64 = t32.astype(np.float64) * DX
    x0 = x64.copy()
    vx = (vth * rng.standard_normal(n)).astype(np.float32)
    dtdx = np.float32(DT / DX)
    kick = np.float32(0.5 * E0 / M_AR * DT)
    kE = np.float32(kick * np.float32(e_field))
    # charge exchange (the ion takes a gas atom's velocity) at the rate n_gas sigma <g>
    p_cx = N_GAS * SIGMA_CX * np.sqrt(16.0 * KB * T_GAS / (np.pi * M_AR)) * DT
    for _ in range(steps):
        vx = vx + kE                      # completing half kick, then the first of the next step
        vx = vx + kE
        t32 = _fma32(vx, dtdx, t32)
        x64 = x64 + vx.astype(np.float64) * DT
        hit = rng.random(n) < p_cx
        k = int(hit.sum())
        if k:
            vx[hit] = (vth * rng.standard_normal(k)).astype(np.float32)
    d32 = t32.astype(np.float64) * DX - x0
    d64 = x64 - x0
    return d32, d64, p_cx


def test_fp32_positions_do_not_bias_ion_drift_or_diffusion():
    d32, d64, p_cx = _transport()
    assert 0.5 < p_cx * 10_000 < 2.0       # about one collision per ion over the run
    drift32, drift64 = d32.mean(), d64.mean()
    var32, var64 = d32.var(), d64.var()
    # the same ions, the same velocities: the differences are the position rounding alone
    # (measured: drift 5e-5, variance 7e-4 relative)
    assert abs(drift32 - drift64) <= 0.01 * abs(drift64), (drift32, drift64)
    assert abs(var32 - var64) <= 0.03 * var64, (var32, var64)
    # per ion, each step rounds by at most half a spacing, 2^-13 cells in this band; a slow
    # ion (|v_x| < 48 m/s) that the rounding keeps in place accumulates close to that bound
    err = np.max(np.abs(d32 - d64)) / DX
    assert err <= 10_000 * 2.0 ** -13
    assert err > 0.1


def test_fp32_positions_field_free_diffusion():
    """Without a field the mean displacement is zero and the spread carries the whole
    effect: quantising the speed in steps q = 97 m/s raises <v^2> by q^2/12, 1.25 % of
    k T / M (measured: +1.35 % in the displacement variance), inside the 3 % moment bound."""
    d32, d64, _ = _transport(n=20_000, steps=10_000, e_field=0.0, seed=1)
    var32, var64 = d32.var(), d64.var()
    assert abs(var32 - var64) <= 0.03 * var64, (var32, var64)
    q = 2.0 ** -12 * DX / DT
    assert abs(var32 / var64 - 1.0 - q * q / 12.0 / (KB * T_GAS / M_AR)) <= 0.006
    assert abs(d32.mean() - d64.mean()) <= 0.01 * np.sqrt(var64)
