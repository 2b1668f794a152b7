"""FP64 CPU oracle of the monolithic FE^2 hot path (test infrastructure).

This package is a plain, slow, obviously correct NumPy/SciPy implementation
of what the GPU library computes, written from the paper (Hesch, Schmidt,
Schuss, "Variational formulation and monolithic solution of computational
homogenization methods", arXiv:2312.12771).  It is test infrastructure only:
the tests, the smoke check and the CPU-baseline leg of the benchmark import
it; the GPU library never does, and the two share no code.  Equation numbers
refer to the paper's sequential numbering.

Modules
-------
tensors   cross product, cofactor, determinant (Sec. 2.1, Eqs. (1)-(2)) and
          the constitutive laws (Eqs. (6)-(8), the Cook law Eq. (59), linear
          isotropic elasticity).
rve       RVE element integration, periodic null-space reduction and static
          condensation (Sec. 3, Eqs. (34)-(35); Sec. 4, Eqs. (39)-(49)).
macro     macro FE, the generalized (monolithic, Sec. 4.2) and classical
          (staggered, Sec. 4.1) Newton schemes, the full block solve
          (Eq. (42)) and the piecewise-constant macro basis of the
          fluctuation.
oned      the 1+1D benchmark of Sec. 5.1: closed form, the six
          discretisations and their L2 errors.
"""
