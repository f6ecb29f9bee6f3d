"""FP64 CPU oracle of the differentiable multigrid solver.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke entry point and the
CPU-baseline leg of the benchmark, never by the GPU library.
"""
