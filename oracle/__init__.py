"""FP64 CPU oracle of the 1D3V PIC/MCC step of Becker et al., arXiv:1608.04601 (Sec. 2.5).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct NumPy
implementation of what the GPU path computes, used to prove the GPU path right.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it; the product path never does, and it shares no code
with the HIP library (it only reads the seeded inputs of ``workloads``).

Every function cites the passage of the paper it follows.  Where the paper is
silent the oracle takes one explicit reading (units, step order, RNG layout, id
assignment, boundary field); each reading is named where it is used.

Pins (tests marked ``not gpu``): Philox against rocRAND's published-definition
implementation; Poisson against the closed form for uniform charge, a dense
solve and Gauss's law; CIC charge and first-moment conservation and exact
linear gather; velocity Verlet against the exact discrete harmonic map and the
constant-field parabola; the null-collision free-flight law and the ion collision
rate against the Maxwellian closed form; collision invariants; Maxwellian
relaxation.  The whole-discharge moments have no closed form: parity unpinned
against the paper (its cross-section data are not available).
"""
from .pic import Oracle, Derived, derive  # noqa: F401
