"""MI355X-native (gfx950) VQE hot path: complex128 state-vector simulation of
the ansatz, Pauli-sum expectation and adjoint gradients behind a C ABI
(include/vqe.h, libvqe.so), with a thin torch binding.

Follows arXiv 2601.09951 (Eqs. 2-7, Algorithm 1).  The HIP library is the
only compute path: importing this package does not load it, but every call
that computes loads libvqe.so and raises if it is missing.
"""
from .capi import VQEError, LibraryMissing  # noqa: F401

__all__ = ["VQEError", "LibraryMissing"]
