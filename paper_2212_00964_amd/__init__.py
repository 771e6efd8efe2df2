"""HEX8 finite-element hot path (residual/tangent assembly, CSR SpMV, Jacobi-Krylov
Newton solves and the adjoint gradient) on AMD Instinct MI355X.

``inputs`` generates seeded synthetic problems; ``fem`` binds the HIP library
``libfem.so`` (import it explicitly: ``from paper_2212_00964_amd import fem``).
"""
from . import inputs  # noqa: F401

__all__ = ["inputs"]
