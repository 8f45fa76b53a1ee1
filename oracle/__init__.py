"""FP64 CPU oracle of the FAR-LIO registration hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The GPU library never links or calls it.
"""
