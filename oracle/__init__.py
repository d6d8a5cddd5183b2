"""FP64 CPU oracle for the overlap operator (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, the smoke check of ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package.  The HIP product path never
imports, links or executes anything here, and nothing here imports it.

* ``oracle.api``   ctypes front end of the plain C implementation
* ``oracle.dense`` NumPy dense-matrix checker for lattices up to 4^4
* ``oracle.build`` compiles ``liboracle.so`` with gcc

Parity pins: every function is pinned by a ``-m "not gpu"`` test against the
paper's printed values, closed forms, invariants or brute force, except the
physics observables the paper reports on its gauge ensemble (not available),
which are not implemented.
"""
