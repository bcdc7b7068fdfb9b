"""FP64 CPU oracle for the shaped-stencil leapfrog acoustic scheme.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the CPU-baseline leg of the benchmark may import this package.  It shares no
code with the HIP library: its stepper is plain C (`fd_oracle.c`), its weights
are exact rationals (`weights.py`), its analytic solutions live in
`analytic.py`.
"""
