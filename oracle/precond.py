"""Basis change between the Hermite-like and the nodal Gauss-Lobatto bases, the
preconditioner of eq. (jacobi) (Section 6.3), and the 1D matrices of eq.
(KDlaplace_dg) (Section 6.4).

Test infrastructure (see oracle/__init__.py).

Conventions.  E_ij = phi^HL_i(x^GL_j) (n x n).  A function with HL
coefficients c^HL has GL coefficients (its values at the GL nodes)
c^GL = E^T c^HL, so c^HL = V c^GL with V = E^-T.  Residuals (dual vectors)
transform with V^T: r^GL = V^T r^HL = T r^HL, T = E^-1.  The preconditioner
of eq. (jacobi) in the HL basis with a diagonal P_d in the GL basis is then
    P^-1 = (T^T x T^T x T^T) P_d^-1 (T x T x T),
applied cell by cell, and A_GL = V_glob^T A_HL V_glob.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import basis as b1d


def hl_to_gl_matrices(k: int):
    """Return E, T = E^-1 and V = E^-T for degree k."""
    hl = b1d.hermite_like(k)
    x = b1d.gauss_lobatto_points(k + 1)
    E = hl.values(x).T            # E[i, j] = phi_i(x_j)
    T = np.linalg.inv(E)
    V = T.T
    return E, T, V


def kron3(M):
    """M x M x M acting on the in-cell index i1 + n i2 + n^2 i3."""
    return np.kron(M, np.kron(M, M))


def cellwise(M3, ncells):
    """Block-diagonal global matrix with the cell block M3."""
    return sp.block_diag([sp.csr_matrix(M3)] * ncells, format="csr")


def apply_cellwise(M3, x, ncells):
    X = np.asarray(x, dtype=np.float64).reshape(ncells, -1)
    return (X @ M3.T).reshape(-1)


def pjacobi_hl(k: int, diag_gl: np.ndarray, r: np.ndarray, ncells: int) -> np.ndarray:
    """P^-1 r of eq. (jacobi) with P_d = diag(A_GL): change the HL residual into
    the GL basis with T^{x3}, scale by the inverse diagonal, and map back with
    (T^T)^{x3}."""
    _, T, _ = hl_to_gl_matrices(k)
    T3 = kron3(T)
    rg = apply_cellwise(T3, r, ncells)
    zg = rg / diag_gl
    return apply_cellwise(T3.T, zg, ncells)


# --------------------------------------------------------------------------
# 1D SIPG stiffness and mass matrices (eq. KDlaplace_dg), global over a
# uniform 1D mesh of `ncell` intervals of length h with mirror boundaries.
# --------------------------------------------------------------------------
def sipg_1d(basis: b1d.Basis1D, ncell: int, h: float, eta: float):
    """Global 1D SIPG matrix L and mass matrix M (cell-wise numbering).

    In 1D the faces are points; with n = +-1 the outward normal, the element
    rows are those of Section 2 with d/dx = (1/h) d/dxi."""
    p = basis.degree
    n = p + 1
    xq, wq = b1d.gauss(p + 1)
    V = basis.values(xq)
    D = basis.derivs(xq) / h
    Kc = D.T @ (wq[:, None] * D) * h
    Mc = V.T @ (wq[:, None] * V) * h
    v0, d0 = basis.values([0.0])[0], basis.derivs([0.0])[0] / h
    v1, d1 = basis.values([1.0])[0], basis.derivs([1.0])[0] / h
    sigma = eta * (p + 1) ** 2 / h
    N = ncell * n
    L = np.zeros((N, N))
    M = np.zeros((N, N))
    for c in range(ncell):
        sl = slice(c * n, (c + 1) * n)
        L[sl, sl] += Kc
        M[sl, sl] += Mc
        # left face (xi = 0, normal -1) and right face (xi = 1, normal +1)
        for (vo, do, nrm, nb, vn, dn) in ((v0, d0, -1.0, c - 1, v1, d1),
                                          (v1, d1, 1.0, c + 1, v0, d0)):
            if 0 <= nb < ncell:
                L[sl, sl] += (sigma * np.outer(vo, vo) - 0.5 * nrm * np.outer(vo, do)
                              - 0.5 * nrm * np.outer(do, vo))
                sn = slice(nb * n, (nb + 1) * n)
                L[sl, sn] += (-sigma * np.outer(vo, vn) - 0.5 * nrm * np.outer(vo, dn)
                              + 0.5 * nrm * np.outer(do, vn))
            else:
                L[sl, sl] += (2 * sigma * np.outer(vo, vo) - nrm * np.outer(vo, do)
                              - nrm * np.outer(do, vo))
    return L, M


def kronecker_cartesian(basis_kind: str, k: int, ncell, h, eta: float):
    """A on a Cartesian brick as  P (M x M x L + M x L x M + L x M x M) P^T
    (eq. KDlaplace_dg applied to the whole mesh), returned in the cell-wise
    numbering.  ncell, h: per-direction cell counts and sizes."""
    bas = b1d.make_basis(basis_kind, k)
    n = k + 1
    Ls, Ms = [], []
    for d in range(3):
        L, M = sipg_1d(bas, ncell[d], h[d], eta)
        Ls.append(L)
        Ms.append(M)
    # Kronecker order: direction 3 slowest, direction 1 fastest
    A = (np.kron(Ms[2], np.kron(Ms[1], Ls[0])) + np.kron(Ms[2], np.kron(Ls[1], Ms[0]))
         + np.kron(Ls[2], np.kron(Ms[1], Ms[0])))
    # permutation from tensor numbering (g1 + N1 (g2 + N2 g3)), g_d = c_d n + i_d,
    # to cell-wise numbering (cell * n^3 + i1 + n i2 + n^2 i3)
    N1, N2, N3 = (ncell[0] * n, ncell[1] * n, ncell[2] * n)
    g3, g2, g1 = np.meshgrid(np.arange(N3), np.arange(N2), np.arange(N1), indexing="ij")
    g1, g2, g3 = g1.ravel(), g2.ravel(), g3.ravel()
    cell = (g1 // n) + ncell[0] * ((g2 // n) + ncell[1] * (g3 // n))
    local = (g1 % n) + n * ((g2 % n) + n * (g3 % n))
    perm = cell * n ** 3 + local            # tensor index -> cell-wise index
    Acw = np.zeros_like(A)
    Acw[np.ix_(perm, perm)] = A
    return Acw
