"""Pins of the oracle's SIPG operator (CPU only).

Each test ties the assembled operator to a property fixed by the paper or by
the mathematics, chosen so that a dropped term, a wrong sign, a wrong index
or a transposed operand fails at least one of them."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import basis as b1d
from oracle import mms, precond
from oracle.sipg import SIPG
from workloads import Mesh, paper_affine_brick, unit_cube

MESHES = {
    "cartesian": unit_cube((3, 2, 2)),
    "deformed": unit_cube((2, 3, 2), 0.1),
    "paper_affine": paper_affine_brick((2, 2, 3)),
}


@pytest.mark.parametrize("mesh_name", list(MESHES))
@pytest.mark.parametrize("basis", ["hermite_like", "nodal_gl"])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_symmetric_positive_definite(mesh_name, basis, k):
    for eta in (1.0, 2.0):
        A = SIPG(MESHES[mesh_name], k, eta, basis).assemble().toarray()
        assert np.max(np.abs(A - A.T)) <= 1e-14 * np.max(np.abs(A)) * 10
        np.linalg.cholesky(A)  # raises if not positive definite


@pytest.mark.parametrize("mesh_name", list(MESHES))
@pytest.mark.parametrize("basis", ["hermite_like", "nodal_gl"])
def test_matrix_free_equals_assembled(mesh_name, basis):
    for k in (2, 4):
        op = SIPG(MESHES[mesh_name], k, 2.0, basis)
        x = np.random.default_rng(3).uniform(-1, 1, op.ndofs)
        y_csr = op.assemble() @ x
        y_mf = op.apply_naive(x)
        assert np.linalg.norm(y_mf - y_csr) <= 1e-14 * np.linalg.norm(y_csr) * 10


@pytest.mark.parametrize("basis", ["hermite_like", "nodal_gl"])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_kronecker_structure_cartesian(basis, k):
    """On a Cartesian brick A = P (M x M x L + M x L x M + L x M x M) P^T with the
    1D SIPG and mass matrices (eq. KDlaplace_dg, applied to the whole mesh);
    non-cubic cells so that every direction has its own h."""
    mesh = Mesh(n=(3, 2, 2), hi=(1.5, 0.8, 1.0))
    A = SIPG(mesh, k, 2.0, basis).assemble().toarray()
    Ak = precond.kronecker_cartesian(basis, k, mesh.n, [0.5, 0.4, 0.5], 2.0)
    assert np.max(np.abs(A - Ak)) <= 1e-14 * np.max(np.abs(A)) * 10


def test_1d_sipg_consistency_and_spd():
    """The 1D matrices used above: L is symmetric positive definite and exact on
    a quadratic that vanishes at both ends (L I_h u = (f, phi) with f = 2)."""
    for k in (2, 3, 5):
        bas = b1d.hermite_like(k)
        ncell, h = 5, 0.2
        L, M = precond.sipg_1d(bas, ncell, h, 2.0)
        assert np.allclose(L, L.T, atol=1e-13)
        np.linalg.cholesky(L)
        np.linalg.cholesky(M)
        pts = b1d.gauss_lobatto_points(k + 1)
        Vb = bas.values(pts)
        xq, wq = b1d.gauss(k + 1)
        u = np.zeros(ncell * (k + 1))
        b = np.zeros_like(u)
        for c in range(ncell):
            x = (c + pts) * h
            u[c * (k + 1):(c + 1) * (k + 1)] = np.linalg.solve(Vb, x * (1 - x))
            b[c * (k + 1):(c + 1) * (k + 1)] = 2.0 * (bas.values(xq).T @ wq) * h
        assert np.max(np.abs(L @ u - b)) < 1e-12


@pytest.mark.parametrize("basis", ["hermite_like", "nodal_gl"])
@pytest.mark.parametrize("k", [2, 3, 4])
def test_consistency_patch(basis, k):
    """SIPG is consistent and Gauss quadrature with k+1 points is exact here, so
    for u = x(1-x)y(1-y)z(1-z) in Q_2 (k >= 2), A I_h u = b(-Laplace u) exactly."""
    op = SIPG(unit_cube((3, 2, 2)), k, 2.0, basis)
    g = lambda x: x * (1 - x)
    u = op_u = mms.interpolate_cartesian_product(op, [g, g, g])
    b = mms.rhs(op, mms.quad_bubble_rhs)
    r = op.assemble() @ u - b
    assert np.max(np.abs(r)) <= 1e-13 * np.max(np.abs(b)) * 10
    assert mms.l2_error(op, op_u, mms.quad_bubble) < 1e-14


@pytest.mark.parametrize("basis", ["hermite_like", "nodal_gl"])
@pytest.mark.parametrize("k", [2, 3])
def test_consistency_patch_graded(basis, k):
    """The same Q_2 patch test on a graded brick (the last cell of every
    direction narrower than the others): the map, the Jacobians and the
    penalty of unequal neighbours reproduce A I_h u = b exactly, and the
    cells tile the unit cube."""
    op = SIPG(Mesh(n=(3, 2, 3), width=(0.4, 0.6, 0.45)), k, 2.0, basis)
    assert abs(op.cell_volume.sum() - 1.0) < 1e-14
    g = lambda x: x * (1 - x)
    u = mms.interpolate_cartesian_product(op, [g, g, g])
    b = mms.rhs(op, mms.quad_bubble_rhs)
    r = op.assemble() @ u - b
    assert np.max(np.abs(r)) <= 1e-13 * np.max(np.abs(b)) * 10
    assert mms.l2_error(op, u, mms.quad_bubble) < 1e-14


@pytest.mark.parametrize("k", [2, 3, 5])
def test_basis_independence(k):
    """Same space and quadrature: A_GL = V^T A_HL V, on a deformed mesh, with the
    GL operator assembled directly in its own basis."""
    mesh = unit_cube((2, 2, 1), 0.1)
    Ah = SIPG(mesh, k, 2.0, "hermite_like").assemble().toarray()
    Ag = SIPG(mesh, k, 2.0, "nodal_gl").assemble().toarray()
    _, T, V = precond.hl_to_gl_matrices(k)
    Vg = np.kron(np.eye(mesh.ncells), precond.kron3(V))
    assert np.max(np.abs(Vg.T @ Ah @ Vg - Ag)) <= 1e-14 * np.max(np.abs(Ag)) * 100


@pytest.mark.parametrize("k", [2, 3, 4])
def test_pjacobi_is_gl_point_jacobi(k):
    """P^-1 of eq. (jacobi) with diag(A_GL) equals GL point-Jacobi mapped back:
    V_glob diag(A_GL)^-1 V_glob^T, and T E = I."""
    mesh = unit_cube((2, 1, 2), 0.1)
    Ag = SIPG(mesh, k, 2.0, "nodal_gl").assemble()
    dg = Ag.diagonal()
    E, T, V = precond.hl_to_gl_matrices(k)
    assert np.allclose(T @ E, np.eye(k + 1), atol=1e-12)
    r = np.random.default_rng(1).uniform(-1, 1, Ag.shape[0])
    z = precond.pjacobi_hl(k, dg, r, mesh.ncells)
    Vg = np.kron(np.eye(mesh.ncells), precond.kron3(V))
    ref = Vg @ ((Vg.T @ r) / dg)
    assert np.max(np.abs(z - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("k", [2, 3])
def test_hermite_like_neighbour_coupling_two_layers(k):
    """Section 4.2: with the Hermite-like basis a cell couples to a face
    neighbour only through the neighbour's value and derivative layers, 2 n^2
    entries, whereas the nodal GL basis couples to the whole neighbour."""
    n = k + 1
    mesh = unit_cube((2, 1, 1), 0.1)
    for basis, layers in (("hermite_like", 2), ("nodal_gl", n)):
        A = SIPG(mesh, k, 2.0, basis).assemble().toarray()
        blk = A[: n ** 3, n ** 3:]            # cell 0 rows, cell 1 columns (x neighbour)
        nz = np.abs(blk) > 1e-13 * np.max(np.abs(A))
        i1 = np.arange(n ** 3) % n
        cols = np.nonzero(nz.any(axis=0))[0]
        rows = np.nonzero(nz.any(axis=1))[0]
        assert set(i1[cols]) == set(range(layers))              # neighbour's low layers
        assert set(i1[rows]) == set(range(n - layers, n))       # own high layers
        assert len(cols) == layers * n * n and len(rows) == layers * n * n


def test_geometry_volumes():
    """Sum of det J w over all cells: 1 on the unit cube (the sine deformation
    fixes the cube's boundary), and det(L) |brick| for the paper's brick."""
    op = SIPG(unit_cube(3, 0.1), 4)
    assert abs(op.cell_volume.sum() - 1.0) < 1e-3
    op = SIPG(unit_cube(4), 2)
    assert abs(op.cell_volume.sum() - 1.0) < 1e-14
    m = paper_affine_brick(2)
    op = SIPG(m, 1)
    vol = np.prod(np.subtract(m.hi, m.lo)) * np.linalg.det(np.array(m.lin))
    assert abs(op.cell_volume.sum() - vol) < 1e-13
    # Cartesian penalty reduces to eta (k+1)^2 / h (Section 2)
    opc = SIPG(unit_cube(4), 3, 2.0)
    assert np.allclose(opc.faces[(0, 1)]["sigma"], 2.0 * 16 / 0.25)


@pytest.mark.parametrize("k", [2, 3])
def test_mms_convergence_cartesian(k):
    """L2 error of the manufactured sine solution decays as h^{k+1}."""
    errs = []
    for nc in (4, 8):
        op = SIPG(unit_cube(nc), k, 2.0)
        A = op.assemble()
        b = mms.rhs(op, mms.sine_rhs)
        u, info = spla.cg(A, b, rtol=1e-13, maxiter=20000)
        assert info == 0
        errs.append(mms.l2_error(op, u, mms.sine))
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - (k + 1)) < 0.15, rate


def test_mms_convergence_deformed():
    errs = []
    for nc in (4, 8):
        op = SIPG(unit_cube(nc, 0.1), 2, 2.0)
        A = op.assemble()
        b = mms.rhs(op, mms.sine_rhs)
        u, info = spla.cg(A, b, rtol=1e-13, maxiter=20000)
        assert info == 0
        errs.append(mms.l2_error(op, u, mms.sine))
    rate = np.log2(errs[0] / errs[1])
    assert rate > 2.7, rate


@pytest.mark.parametrize("k", [1, 2, 4])
def test_nodal_gauss_basis_same_space(k):
    """The nodal Gauss basis (Section 4.1, S = I) spans the same space: with
    E_ij = phi^HL_i(x^Gauss_j), A_Gauss = V^T A_HL V for V = E^-T, on a deformed
    mesh; the Gauss operator is SPD and its matrix-free product equals CSR."""
    mesh = unit_cube((2, 1, 2), 0.1)
    Ah = SIPG(mesh, k, 2.0, "hermite_like").assemble().toarray()
    opg = SIPG(mesh, k, 2.0, "nodal_gauss")
    Ag = opg.assemble().toarray()
    xg, _ = b1d.gauss(k + 1)
    E = b1d.hermite_like(k).values(xg).T            # E[i, j] = phi_i(x_j)
    V = np.linalg.inv(E).T
    Vg = np.kron(np.eye(mesh.ncells), precond.kron3(V))
    assert np.max(np.abs(Vg.T @ Ah @ Vg - Ag)) <= 1e-13 * np.max(np.abs(Ag))
    np.linalg.cholesky(Ag)
    x = np.random.default_rng(k).uniform(-1, 1, opg.ndofs)
    assert np.allclose(opg.apply_naive(x), Ag @ x, rtol=0, atol=1e-13 * np.abs(Ag @ x).max())
