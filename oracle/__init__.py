"""Plain FP64 CPU oracle for the Newton step of the paper's interior-point
method (problem (1), KKT system (2)).

TEST INFRASTRUCTURE ONLY: it exists to check the device library.  Only the
tests, the smoke check and the CPU-baseline leg of the benchmark may import
it; the product package never does, and the two share no code.
"""
