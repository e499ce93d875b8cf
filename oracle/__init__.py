"""Plain FP64 CPU oracle of the volumetric lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of bench.py, never by the product package.
"""
