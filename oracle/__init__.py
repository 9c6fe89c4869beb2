"""FP64 CPU oracle for the SIPG Laplacian in the Hermite-like basis.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the HIP path: every step here is
written independently, in plain NumPy/SciPy, in float64, and follows the
paper's definitions:

  * basis.py     1D bases (Hermite-like of Section 4.1 and Appendix A,
                 nodal Gauss-Lobatto Lagrange, the rejected classical Hermite
                 and Hermite+Legendre bases used only as Table 1 pins),
                 Gauss quadrature, mass-matrix condition numbers.
  * mesh.py      reference-to-physical maps, Jacobians, cell volumes.
  * sipg.py      explicit assembly of A_ij = a_h(phi_j, phi_i) for the weak
                 form of Section 2 (CSR), and a naive matrix-free product
                 (dense per-cell evaluation matrices, no sum factorization).
  * precond.py   basis-change matrices and the preconditioner of eq. (jacobi)
                 in Section 6.3; 1D SIPG/mass matrices of eq. (KDlaplace_dg).
  * mms.py       manufactured solution, right-hand side, interpolation, L2
                 error.

Pins (tests/test_oracle_*.py, marked "not gpu") tie every function to what the
paper or the mathematics fixes: Appendix A closed forms, the Figure 2 p=7
constants, Table 1 condition numbers, the face property, symmetry and
positive definiteness, the Kronecker structure on Cartesian meshes, exact
consistency for quadratics, basis independence, and O(h^{k+1}) convergence.
"""
