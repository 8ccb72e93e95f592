"""Reference (oracle) implementation of the tensorized approximation of the
long-range two-electron integrals, and exact-integral references used to pin it.

This package is TEST INFRASTRUCTURE.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it.  The GPU library never
imports, links or calls anything here, and nothing here imports the GPU
library: the two share no code.

Modules
-------
tairef  the method itself, step by step, in plain FP64 numpy.
exact   closed forms and brute-force integrals that the method approximates.
"""
