"""Chebyshev-filtered subspace iteration for the plane-wave generalized eigenproblem on MI355X.

Modules: ``chebfd`` (binding of libchebfd.so), ``driver`` (outer loop), ``workload`` (seeded synthetic
inputs), ``build`` (hipcc build of the library). Importing the package loads nothing; the library is
loaded on first use by ``chebfd.load_library``.
"""
