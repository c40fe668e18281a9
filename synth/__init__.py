"""Seeded synthetic inputs: meshes, deformations and material parameters.

Shared by the oracle tests, the GPU parity tests and the benchmark.  Holds no
strain-energy or force arithmetic of the method itself.
"""
