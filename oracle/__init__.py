"""Plain FP64 CPU oracle of the algebraic domain-decomposition method.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's
CPU-baseline leg may import it; the product path (the HIP library and its
Python binding) never does, and shares no code with it.
"""
