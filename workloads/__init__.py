"""Seeded synthetic problem definitions shared by the oracle and the GPU tests.

This package holds problem *data* only: coefficient fields, manufactured
solutions and their forcing, and the seeded random draws that pick them.
It contains none of the discretisation or of the iHDG arithmetic, so that the
oracle and the HIP path, which both read it, stay independent.
"""
from .problems import *  # noqa: F401,F403
