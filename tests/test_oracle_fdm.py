"""Pins of the oracle's block-Jacobi (fast diagonalization) preconditioner
of Section 6.4 (CPU only).

The separable block of eq. (KDlaplace_dg) is tied to the independently
assembled 3D operator: on a Cartesian brick the diagonal block of every
interior cell must equal it exactly, while cells at the boundary (different
mirror weights, neglected as in the paper) must differ."""
import numpy as np
import pytest

from oracle import fdm
from oracle.sipg import SIPG
from workloads import Mesh, paper_affine_brick, unit_cube

# anisotropic cells (h = 0.25, 1/3, 0.2) so that a swapped direction fails
BRICK = Mesh(n=(3, 3, 4), lo=(0.0, 0.0, 0.0), hi=(0.75, 1.0, 0.8))


def _diag_block(A, c, n3):
    return A[c * n3:(c + 1) * n3, c * n3:(c + 1) * n3].toarray()


def _interior_cells(mesh):
    nx, ny, nz = mesh.n
    return [ix + nx * (iy + ny * iz) for iz in range(1, nz - 1) for iy in range(1, ny - 1)
            for ix in range(1, nx - 1)]


@pytest.mark.parametrize("basis", ["hermite_like", "nodal_gl"])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_block_equals_interior_cell_block_of_assembled_operator(basis, k):
    for eta in ((1.0, 2.0) if k <= 2 else (2.0,)):
        A = SIPG(BRICK, k, eta, basis).assemble()
        n3 = (k + 1) ** 3
        hs = fdm.cell_lengths(BRICK)
        for c in _interior_cells(BRICK):
            P = fdm.block(basis, k, eta, hs[c])
            Akk = _diag_block(A, c, n3)
            assert np.max(np.abs(P - Akk)) <= 1e-13 * np.max(np.abs(Akk)), (basis, k, eta, c)


@pytest.mark.parametrize("k", [1, 3, 4])
def test_boundary_cells_differ_from_the_assembled_block(k):
    """The interior-element matrices are used at the boundary too (Section
    6.4): the corner cell's block is not reproduced."""
    A = SIPG(BRICK, k, 2.0).assemble()
    n3 = (k + 1) ** 3
    P = fdm.block("hermite_like", k, 2.0, fdm.cell_lengths(BRICK, [0])[0])
    Akk = _diag_block(A, 0, n3)
    assert np.max(np.abs(P - Akk)) > 1e-3 * np.max(np.abs(Akk))


@pytest.mark.parametrize("k", [2, 4])
def test_apply_is_exact_inverse_on_interior_cells(k):
    A = SIPG(BRICK, k, 2.0).assemble()
    n3 = (k + 1) ** 3
    r = np.random.default_rng(k).uniform(-1, 1, BRICK.ncells * n3)
    z = fdm.apply(BRICK, k, 2.0, "hermite_like", r).reshape(BRICK.ncells, n3)
    R = r.reshape(BRICK.ncells, n3)
    for c in _interior_cells(BRICK):
        ref = np.linalg.solve(_diag_block(A, c, n3), R[c])
        assert np.linalg.norm(z[c] - ref) <= 1e-12 * np.linalg.norm(ref)


def test_block_is_symmetric_positive_definite():
    for basis in ("hermite_like", "nodal_gl"):
        for k in (1, 3, 6):
            P = fdm.block(basis, k, 2.0, (0.3, 0.7, 0.45))
            assert np.max(np.abs(P - P.T)) <= 1e-14 * np.max(np.abs(P)) * 10
            np.linalg.cholesky(P)


def test_cell_lengths_closed_forms():
    # affine brick: J = L diag(h), so h_d = h_d |L e_d|
    mesh = paper_affine_brick((4, 3, 2))
    h = (np.array(mesh.hi) - np.array(mesh.lo)) / np.array(mesh.n)
    Lm = np.array(mesh.lin)
    ref = h * np.linalg.norm(Lm, axis=0)
    hs = fdm.cell_lengths(mesh)
    assert np.allclose(hs, ref[None, :], rtol=1e-15, atol=0)
    # Cartesian: the cell extents
    assert np.allclose(fdm.cell_lengths(BRICK), [0.25, 1 / 3, 0.2], rtol=1e-15)
    # deformed: at the cell centre (1/2,1/2,1/2) of the single-cell unit cube
    # the deformation gradient is I + a (1,1,1) grad s with grad s = 0 there
    assert np.allclose(fdm.cell_lengths(unit_cube(1, 0.1)), [1.0, 1.0, 1.0], rtol=1e-15)
