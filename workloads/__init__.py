"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle harness.

This package generates *inputs only*: periodic tetrahedral meshes, material
fields as closed-form functions of position, source/receiver positions and
serving request streams.  It holds none of the discretisation's arithmetic
(no basis, no quadrature, no operator), so both the HIP library and the FP64
oracle can consume what it produces without sharing any method code.
"""
from .mesh import kuhn_periodic_mesh  # noqa: F401
from . import media  # noqa: F401
