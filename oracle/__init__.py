"""FP64 CPU oracle for the GMMNLSE massively parallel algorithm.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg.  Never imported by the product package.
"""
