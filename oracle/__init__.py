"""CPU FP64 oracle for the second-order adjoint quantum-control path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py``.  The product package never imports it, and the two
share no code beyond the seeded input generators in ``paper_2505_00529_amd.inputs``.

Parity status: every function here is pinned by ``tests/test_oracle_pins.py`` (closed
forms, invariants, library routines, finite differences, 50-digit brute force).
"""
from .qoc_oracle import *  # noqa: F401,F403
