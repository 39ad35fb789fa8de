"""CPU FP64 oracle of the background-field PSFD / Lippmann-Schwinger solver.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports, links or calls
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may use it. It shares no code with the HIP library; both
are fed from the seeded input generators in ``paper_2606_25541_amd.clips``,
which contain no solver arithmetic.

Everything here is plain NumPy/SciPy in float64/complex128, written step by step
from the paper (vector Helmholtz eq. (1), background decomposition eqs. (2)-(3),
outer fixed point eqs. (8)-(9), Lippmann-Schwinger eqs. (11)-(12), windowed
dyadic Green's function eqs. (13)-(17), discrete system eq. (18)) plus the
readings listed in the design notes for the points where the paper is silent.

``oracle.isolated`` holds the spherically windowed dyadic kernel of the
isolated-domain mode (eqs. (15)-(17) with the corrected h and A(0)), pinned by a
radial quadrature of the windowed kernel, and the isolated apply with the
4x-oversampled kernel precompute; it is not on the periodic hot path.

Parity status: every function is pinned by the ``-m "not gpu"`` tests
(quadrature of the kernel, independent transfer-matrix code, dense direct
solves, reciprocity, uniform-film convergence to the layered reflection, Born
limit, energy balance, finite differences for the adjoint).
"""
from .psfd import *  # noqa: F401,F403
