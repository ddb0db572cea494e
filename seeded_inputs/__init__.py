"""Seeded synthetic inputs (lattice vectors, shifts, problems, kinematics).

Shared by the oracle and the GPU path; holds none of the method's
arithmetic.
"""
