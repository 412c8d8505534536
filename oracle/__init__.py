"""FP64 CPU oracle of the coupled LB / rigid-ellipsoid step.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU-baseline leg).
"""
