"""FP64 CPU oracle of the adjoint Monte Carlo method (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It shares no code with the GPU library.
"""
