"""Independent CPU oracle for the adaptive SpMV path.  TEST INFRASTRUCTURE.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import anything from this package.  The GPU library
never calls it, and it shares no code, header, table or constant with the GPU
sources; the only thing both sides consume is the seeded input generator
module ``paper_1210_2536_amd.synth``, which holds none of the method's
arithmetic.

Contents (each module cites the part of the paper it follows):

* ``spmv``      y = A x in float64, accurate (compensated) and plain modes
                (C library ``ref_spmv.c``).
* ``convert``   CSR <-> COO / ELL / DIA layouts, bit-exact (Section 2.1).
* ``features``  the Table 3 parameters plus the selector's 12 inputs
                (Section 4).
* ``rules``     the rule-based format choice built from the thresholds of
                Section 4 in the Section 6 order.
* ``mlp``       float64 forward / backward / Adam of the selector network.
* ``amortize``  the break-even call count of Equation 2.
"""
