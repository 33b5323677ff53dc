"""FP64 CPU oracle for the galaxy-fitting hot path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the GPU package.
"""
