"""CPU FP64 oracle of the diffuse-interface MRT lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
baseline of the benchmark, never by the product package.
"""
