"""Pins of the oracle's cloud-in-cell weighting, Poisson solve and node field
(Sec. 2 Eq. (poisson); Sec. 2.2 boundary values; Sec. 2.5 cloud-in-cell)."""
import numpy as np
import pytest

from oracle import field
from oracle.constants import EPS0


@pytest.mark.parametrize("n", [2, 3, 16, 128, 4096])
@pytest.mark.parametrize("phi0", [0.0, 100.0, -37.5])
def test_poisson_uniform_charge_closed_form(n, phi0):
    """Uniform rho: phi(x) = phi0 (1 - x/d) + rho x (d - x)/(2 eps0), exact at the nodes
    (central differences are exact for quadratics); boundary fields exact too."""
    d = 0.025
    dx = d / n
    rho = 3.0e-4  # C/m^3
    Q = np.full(n + 1, rho * dx)
    Q[0] = Q[-1] = rho * dx / 2
    x = np.arange(n + 1) * dx
    phi = field.solve_poisson(Q, dx, phi0, 0.0)
    exact = phi0 * (1 - x / d) + rho * x * (d - x) / (2 * EPS0)
    scale = max(abs(phi0), np.abs(exact).max())
    assert np.allclose(phi, exact, rtol=0, atol=1e-11 * scale)
    E = field.node_field(phi, Q, dx)
    E_exact = phi0 / d - rho * (d - 2 * x) / (2 * EPS0)
    assert np.allclose(E, E_exact, rtol=0, atol=1e-9 * np.abs(E_exact).max())


def test_poisson_matches_dense_solve():
    rng = np.random.default_rng(1)
    for n in (2, 5, 33):
        dx = 0.01 / n
        Q = rng.normal(size=n + 1) * 1e-9
        phi0, phiN = rng.normal() * 50, 0.0
        A = np.zeros((n + 1, n + 1))
        b = np.zeros(n + 1)
        A[0, 0] = A[n, n] = 1.0
        b[0], b[n] = phi0, phiN
        for i in range(1, n):
            A[i, i - 1], A[i, i], A[i, i + 1] = -1.0 / dx ** 2, 2.0 / dx ** 2, -1.0 / dx ** 2
            b[i] = Q[i] / (EPS0 * dx)
        ref = np.linalg.solve(A, b)
        got = field.solve_poisson(Q, dx, phi0, phiN)
        assert np.allclose(got, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_gauss_law_surface_charges():
    """sigma_0 + sigma_d + sum Q = 0 for any charge and any applied voltage."""
    rng = np.random.default_rng(2)
    n, d = 64, 0.02
    dx = d / n
    for _ in range(5):
        Q = rng.normal(size=n + 1) * 1e-8
        phi = field.solve_poisson(Q, dx, rng.normal() * 100, 0.0)
        E = field.node_field(phi, Q, dx)
        total = EPS0 * E[0] - EPS0 * E[-1] + Q.sum()
        assert abs(total) < 1e-12 * np.abs(Q).sum()


def test_cic_conservation_and_node_exactness():
    rng = np.random.default_rng(3)
    n, d = 50, 0.02
    dx = d / n
    x = rng.uniform(0, d, 10_000)
    q = rng.normal(size=x.size)
    Q = field.deposit(x, q, dx, n)
    nodes = np.arange(n + 1) * dx
    assert np.isclose(Q.sum(), q.sum(), rtol=1e-12, atol=1e-9)
    assert np.isclose((Q * nodes).sum(), (q * x).sum(), rtol=1e-10, atol=1e-12)  # first moment
    # a particle on a node deposits only there; the last cell includes x = d
    Q1 = field.deposit(np.array([7 * dx]), 1.0, dx, n)
    assert Q1[7] == 1.0 and Q1.sum() == 1.0
    Q2 = field.deposit(np.array([d]), 1.0, dx, n)
    assert Q2[n] == 1.0 and Q2.sum() == 1.0


def test_linear_gather_exact():
    rng = np.random.default_rng(4)
    n, d = 40, 0.03
    dx = d / n
    nodes = np.arange(n + 1) * dx
    E = 5.0 + 1234.0 * nodes
    x = rng.uniform(0, d, 1000)
    assert np.allclose(field.gather(E, x, dx, n), 5.0 + 1234.0 * x, rtol=1e-12)
