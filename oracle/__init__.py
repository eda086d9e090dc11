"""Plain FP64 CPU oracle of the VLBM time step, exact solutions and the
reference adjoint.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product library never does.
"""
