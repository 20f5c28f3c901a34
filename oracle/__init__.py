"""FP64 CPU oracle of the rational-Arnoldi FRF sweep.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the CPU-baseline leg
of the benchmark. The product path (the HIP library and its binding) never imports it.
"""
