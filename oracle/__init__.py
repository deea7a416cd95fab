"""FP64 reference implementations for 1WQC pattern execution.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library ``paper_1604_05659_amd`` and is never on its path.

* ``oracle.core``      -- ctypes wrapper of the complex128 C oracle
                          (``owqs_oracle.c``): elimination-based execution.
* ``oracle.proa``      -- pattern reordering (PROA, Sec. 4.3, Eq. 18).
* ``oracle.substates`` -- sub-state execution: one vector per group of
                          entangled qubits, merged by tensor product on E
                          (Sec. 4.1, Sec. 4.4.1, Fig. 8).
* ``oracle.gflow``     -- generalised flow of a pattern's open graph by
                          exhaustive search (the EOWQS premise, Sec. 4.5).
* ``oracle.reference`` -- independent numpy references: a full-tensor brute
                          force with projectors and no elimination, and a
                          J/CZ circuit simulator.
"""
