"""FP64 CPU oracle for the batched segment-QP path (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It shares no code with the HIP library.
"""
