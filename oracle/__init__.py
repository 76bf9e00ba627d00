"""Plain FP64 CPU oracle of PCBA and exact-rational Bernstein checks.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The HIP library never imports or links it, and
it never imports the HIP library.
"""
