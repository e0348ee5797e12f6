"""CPU oracle for the AtA Gram product (arXiv 2110.13042).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the library and its Python
binding never do, and nothing here imports them.

* ``plain``     -- O1, the plain FP64 definition C = A^T A (C code, OpenMP).
* ``recursive`` -- O2, the recursive AtA / Strassen algorithm of Sec. 3 written
                   out step by step in FP64, with operation counters.
* ``emulate``   -- CPU emulation of the reduced-precision leaf arithmetic
                   (split-BF16, block-scaled FP8), column-norm spread flags and
                   the Freivalds residual probe.

Parity status of each function is recorded in its docstring; a function with
no independent pin says "parity unpinned".
"""
