"""CPU reference (oracle) for the direct Monte Carlo parameter scan.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product path never imports it.
"""
