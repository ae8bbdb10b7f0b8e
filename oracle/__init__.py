"""Brute-force CPU oracle for ensemble KSG transfer entropy.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg.  It shares no code with the GPU library.
"""
