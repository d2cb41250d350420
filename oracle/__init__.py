"""Plain FP64 CPU oracle for the MGRIT space-fractional diffusion solver.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark.  It shares no code with the HIP path and
the product path never imports it.
"""
