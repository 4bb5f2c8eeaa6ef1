"""Cloud-in-cell weighting, the Poisson solve and the node field.

Sec. 2.5: particles are cloud-in-cell, their weight to the grid falling linearly from
the particle to the two nearest nodes (deposit and gather alike).
Sec. 2, Eq. (poisson): -d^2 phi/dz^2 = (e0/eps0)(n_i - n_e).
Sec. 2.2: phi(0, t) = V0 sin(2 pi f t), phi(d, t) = 0.
Sec. 2.3: second-order central differences for Poisson (stated for the fluid codes;
read here as the PIC discretisation too).

Readings: N_c cells and N_c + 1 nodes x_i = i dx; a particle in cell
j = min(floor(x/dx), N_c - 1) gives (1 - w) to node j and w to node j + 1 with
w = x/dx - j.  Q_i is the node charge per electrode area [C/m^2].  The interior field
is the central difference of phi; the two boundary fields follow from Gauss's law over
the half cell next to each electrode.
"""
import numpy as np
from scipy.linalg import solve_banded

from .constants import EPS0


def cic(x, dx, n_cells):
    t = np.asarray(x, dtype=np.float64) / dx
    j = np.minimum(np.floor(t), n_cells - 1).astype(np.int64)
    return j, t - j


def deposit(x, charge, dx, n_cells):
    """Node charges: sum over particles of charge * CIC weight (charge scalar or per particle)."""
    j, w = cic(x, dx, n_cells)
    q = np.broadcast_to(np.asarray(charge, dtype=np.float64), j.shape)
    n = n_cells + 1
    return (np.bincount(j, weights=q * (1.0 - w), minlength=n)
            + np.bincount(j + 1, weights=q * w, minlength=n))


def gather(E_nodes, x, dx, n_cells):
    j, w = cic(x, dx, n_cells)
    return (1.0 - w) * E_nodes[j] + w * E_nodes[j + 1]


def solve_poisson(Q, dx, phi0, phiN):
    """phi at the nodes from -(phi_{i-1} - 2 phi_i + phi_{i+1})/dx^2 = Q_i/(eps0 dx), i = 1..N_c-1."""
    n = Q.shape[0] - 1
    phi = np.empty(n + 1)
    phi[0], phi[n] = phi0, phiN
    if n == 1:
        return phi
    rhs = dx * Q[1:n] / EPS0
    rhs[0] += phi0
    rhs[-1] += phiN
    ab = np.zeros((3, n - 1))
    ab[0, 1:] = -1.0
    ab[1, :] = 2.0
    ab[2, :-1] = -1.0
    phi[1:n] = solve_banded((1, 1), ab, rhs)
    return phi


def node_field(phi, Q, dx):
    """E_i = (phi_{i-1} - phi_{i+1})/(2 dx) inside; E_0 = (phi_0 - phi_1)/dx - Q_0/eps0 and
    E_N = (phi_{N-1} - phi_N)/dx + Q_N/eps0 by Gauss's law over the boundary half cells."""
    E = np.empty_like(phi)
    E[1:-1] = (phi[:-2] - phi[2:]) / (2.0 * dx)
    E[0] = (phi[0] - phi[1]) / dx - Q[0] / EPS0
    E[-1] = (phi[-2] - phi[-1]) / dx + Q[-1] / EPS0
    return E
