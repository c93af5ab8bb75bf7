"""FP64 CPU oracle for the MLS-MPM step (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP path.
"""
