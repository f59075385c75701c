"""TEST INFRASTRUCTURE ONLY: the plain complex128 CPU oracle (oracle.c via
oracle.py) and the brute-force full-unitary checker (fullmatrix.py). Only
tests, the smoke check and the benchmark's CPU-baseline leg may use it."""
