"""MI355X-native hot path of the Adam-based AC unit-commitment solver
(Chevalier, "A Parallelized, Adam-Based Solver for Reserve and Security
Constrained AC Unit Commitment", PSCC 2024).

Importing the package loads nothing native; ``paper_2310_06650_amd.qg`` binds
the HIP library and raises if it has not been built.
"""
