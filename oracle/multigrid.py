"""Nested-space embeddings used to check the multigrid transfers: between a
brick and its coarsening by two (h), and between degrees on one mesh (p).

Test infrastructure (see oracle/__init__.py).  A coarse cell of a brick is
split into 2 x 2 x 2 children; on child side s of a direction the coarse 1D
function phi_j((s + xi) / 2) is again a polynomial of degree k in xi, so it
has exact coefficients in the fine basis.  The prolongation of a coarse
vector is this change of representation on every child, and the restriction
is its transpose.
"""
from __future__ import annotations

import numpy as np

from . import basis as b1d
from .mesh import cell_bounds


def child_embedding(kind: str, k: int):
    """M_s[i, j] with phi_j((s + xi)/2) = sum_i M_s[i, j] phi_i(xi), s = 0, 1.
    Computed by least squares on k + 4 Gauss points (exact: polynomials)."""
    bas = b1d.make_basis(kind, k)
    x, _ = b1d.gauss(k + 4)
    V = bas.values(x)                                   # [m, i]
    out = []
    for s in (0, 1):
        C = bas.values(0.5 * (s + x))                   # [m, j]
        M, *_ = np.linalg.lstsq(V, C, rcond=None)
        out.append(M)
    return out


def prolongate(coarse: np.ndarray, nc_fine, kind: str, k: int) -> np.ndarray:
    """Fine-mesh coefficients of a coarse-mesh function (cell-wise layout)."""
    n = k + 1
    M = child_embedding(kind, k)
    fx, fy, fz = nc_fine
    cx, cy, cz = fx // 2, fy // 2, fz // 2
    C = np.asarray(coarse, dtype=np.float64).reshape(cz, cy, cx, n ** 3)
    F = np.zeros((fz, fy, fx, n ** 3))
    for s3 in (0, 1):
        for s2 in (0, 1):
            for s1 in (0, 1):
                P = np.kron(M[s3], np.kron(M[s2], M[s1]))
                F[s3::2, s2::2, s1::2] = C @ P.T
    return F.reshape(-1)


def restrict(fine: np.ndarray, nc_fine, kind: str, k: int) -> np.ndarray:
    n = k + 1
    M = child_embedding(kind, k)
    fx, fy, fz = nc_fine
    cx, cy, cz = fx // 2, fy // 2, fz // 2
    F = np.asarray(fine, dtype=np.float64).reshape(fz, fy, fx, n ** 3)
    C = np.zeros((cz, cy, cx, n ** 3))
    for s3 in (0, 1):
        for s2 in (0, 1):
            for s1 in (0, 1):
                P = np.kron(M[s3], np.kron(M[s2], M[s1]))
                C += F[s3::2, s2::2, s1::2] @ P
    return C.reshape(-1)


def degree_embedding(kind: str, kf: int, kc: int):
    """E[i, j] with phi^{kc}_j(xi) = sum_i E[i, j] phi^{kf}_i(xi) (kc <= kf):
    the degree-kc space is a subspace of the degree-kf one.  Least squares on
    kf + 4 Gauss points (exact: polynomials of degree kf)."""
    bf = b1d.make_basis(kind, kf)
    bc = b1d.make_basis(kind, kc)
    x, _ = b1d.gauss(kf + 4)
    E, *_ = np.linalg.lstsq(bf.values(x), bc.values(x), rcond=None)
    return E


def p_prolongate(coarse: np.ndarray, ncells: int, kind: str, kf: int, kc: int) -> np.ndarray:
    """Degree-kf coefficients of a degree-kc function, cell by cell."""
    E = degree_embedding(kind, kf, kc)
    P = np.kron(E, np.kron(E, E))
    return (np.asarray(coarse, dtype=np.float64).reshape(ncells, (kc + 1) ** 3) @ P.T).reshape(-1)


def p_restrict(fine: np.ndarray, ncells: int, kind: str, kf: int, kc: int) -> np.ndarray:
    E = degree_embedding(kind, kf, kc)
    P = np.kron(E, np.kron(E, E))
    return (np.asarray(fine, dtype=np.float64).reshape(ncells, (kf + 1) ** 3) @ P).reshape(-1)


# ---------------------------------------------------------------------------
# Nested bricks in general (graded coarse levels): each fine cell lies inside
# one coarse cell in every direction, at some sub-interval of it.
# ---------------------------------------------------------------------------
def interval_embeddings(kind: str, k: int, fine_bounds, coarse_bounds):
    """For each fine cell [a, b] of one direction: the coarse cell [A, B] that
    contains it and M with phi_j((a + xi (b - a) - A) / (B - A)) =
    sum_i M[i, j] phi_i(xi) (least squares on k + 4 Gauss points, exact)."""
    bas = b1d.make_basis(kind, k)
    x, _ = b1d.gauss(k + 4)
    V = bas.values(x)
    out = []
    for i in range(len(fine_bounds) - 1):
        a, b = float(fine_bounds[i]), float(fine_bounds[i + 1])
        I = int(np.searchsorted(coarse_bounds, 0.5 * (a + b))) - 1
        A, B = float(coarse_bounds[I]), float(coarse_bounds[I + 1])
        tol = 1e-13 * (B - A)
        if not (A - tol <= a and b <= B + tol):
            raise ValueError("the fine brick is not nested in the coarse one")
        M, *_ = np.linalg.lstsq(V, bas.values((a + x * (b - a) - A) / (B - A)), rcond=None)
        out.append((I, M))
    return out


def prolongate_nested(coarse: np.ndarray, fine_mesh, coarse_mesh, kind: str, k: int) -> np.ndarray:
    """Fine-brick coefficients of a coarse-brick function, for any pair of
    nested bricks (cell-wise layout, x fastest)."""
    n3 = (k + 1) ** 3
    emb = [interval_embeddings(kind, k, cell_bounds(fine_mesh, d), cell_bounds(coarse_mesh, d)) for d in range(3)]
    fx, fy, fz = fine_mesh.n
    cx, cy, cz = coarse_mesh.n
    C = np.asarray(coarse, dtype=np.float64).reshape(cz, cy, cx, n3)
    F = np.zeros((fz, fy, fx, n3))
    for kz in range(fz):
        Iz, Mz = emb[2][kz]
        for ky in range(fy):
            Iy, My = emb[1][ky]
            for kx in range(fx):
                Ix, Mx = emb[0][kx]
                F[kz, ky, kx] = np.kron(Mz, np.kron(My, Mx)) @ C[Iz, Iy, Ix]
    return F.reshape(-1)


def restrict_nested(fine: np.ndarray, fine_mesh, coarse_mesh, kind: str, k: int) -> np.ndarray:
    """Transpose of prolongate_nested."""
    n3 = (k + 1) ** 3
    emb = [interval_embeddings(kind, k, cell_bounds(fine_mesh, d), cell_bounds(coarse_mesh, d)) for d in range(3)]
    fx, fy, fz = fine_mesh.n
    cx, cy, cz = coarse_mesh.n
    F = np.asarray(fine, dtype=np.float64).reshape(fz, fy, fx, n3)
    C = np.zeros((cz, cy, cx, n3))
    for kz in range(fz):
        Iz, Mz = emb[2][kz]
        for ky in range(fy):
            Iy, My = emb[1][ky]
            for kx in range(fx):
                Ix, Mx = emb[0][kx]
                C[Iz, Iy, Ix] += np.kron(Mz, np.kron(My, Mx)).T @ F[kz, ky, kx]
    return C.reshape(-1)
