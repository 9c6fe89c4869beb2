"""Element-wise block-Jacobi preconditioner of Section 6.4 (fast
diagonalization), the plain definition.

Test infrastructure (see oracle/__init__.py).

On a Cartesian cell the SIPG cell matrix is the Kronecker sum of eq.
(KDlaplace_dg),
    P_K = M_3 (x) M_2 (x) L_1 + M_3 (x) L_2 (x) M_1 + L_3 (x) M_2 (x) M_1,
with L_d the 1D SIPG stiffness matrix of an element whose two neighbours are
interior (eq. discrete_laplace in 1D, own-own rows) and M_d the 1D mass
matrix, both on an interval of length h_d.  The rightmost factor acts on the
fastest in-cell index i1 (direction x).  As in Section 6.4, the interior
element matrices are used for every cell, also for cells at the boundary.

Reading for cells that are not axis-aligned boxes (the paper refers to other
work): h_d = |J(centre) e_d|, the length of the image of the reference edge
direction e_d at the cell centre; this is exact on Cartesian cells.

The oracle forms P_K explicitly (n^3 x n^3, numpy.kron) and solves with it;
the eigen-decomposition that the device code uses is not involved.
"""
from __future__ import annotations

import numpy as np

from . import basis as b1d
from .mesh import map_points
from .precond import sipg_1d


def interior_1d(basis_kind: str, k: int, h: float, eta: float):
    """(L, M) of the middle element of a three-element 1D SIPG mesh with
    element length h: the element matrix of a cell with two interior faces."""
    n = k + 1
    L, M = sipg_1d(b1d.make_basis(basis_kind, k), 3, h, eta)
    sl = slice(n, 2 * n)
    return L[sl, sl].copy(), M[sl, sl].copy()


def cell_lengths(mesh, cells=None) -> np.ndarray:
    """[C, 3]: h_d = |J(1/2, 1/2, 1/2) e_d| per cell."""
    if cells is None:
        cells = np.arange(mesh.ncells)
    _, J = map_points(mesh, np.asarray(cells), np.array([[0.5, 0.5, 0.5]]))
    return np.linalg.norm(J[:, 0], axis=1)          # column norms: |J e_d|


def block(basis_kind: str, k: int, eta: float, hs) -> np.ndarray:
    """P_K of eq. (KDlaplace_dg) for cell lengths hs = (h_1, h_2, h_3)."""
    L1, M1 = interior_1d(basis_kind, k, float(hs[0]), eta)
    L2, M2 = interior_1d(basis_kind, k, float(hs[1]), eta)
    L3, M3 = interior_1d(basis_kind, k, float(hs[2]), eta)
    return (np.kron(M3, np.kron(M2, L1)) + np.kron(M3, np.kron(L2, M1))
            + np.kron(L3, np.kron(M2, M1)))


def apply(mesh, k: int, eta: float, basis_kind: str, r: np.ndarray) -> np.ndarray:
    """z_K = P_K^-1 r_K for every cell (cell-wise layout)."""
    n3 = (k + 1) ** 3
    hs = cell_lengths(mesh)
    R = np.asarray(r, dtype=np.float64).reshape(mesh.ncells, n3)
    Z = np.empty_like(R)
    cache = {}
    for c in range(mesh.ncells):
        key = tuple(np.round(hs[c], 15))
        if key not in cache:
            cache[key] = block(basis_kind, k, eta, hs[c])
        Z[c] = np.linalg.solve(cache[key], R[c])
    return Z.reshape(-1)
