"""FP64 CPU oracle of the EM-PIC step -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It shares no code with the HIP path.
"""
