"""GPU parity of the tensor-product basis change, the GL diagonal and the
preconditioner of eq. (jacobi) against the oracle."""
import numpy as np
import pytest

from oracle import precond
from oracle.sipg import SIPG
from workloads import unit_cube, paper_affine_brick, uniform_vector
from tests.gpu_util import banner, rel_errors, require_gpu

pytestmark = pytest.mark.gpu


def _dev(torch, x, dtype):
    return torch.from_numpy(np.asarray(x)).to(device="cuda", dtype=torch.float64 if dtype == "f64" else torch.float32)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_basis_change_modes(k, dtype):
    torch, P = require_gpu()
    banner(f"basis change k={k} {dtype}")
    mesh = unit_cube((3, 2, 4))
    ncells = mesh.ncells
    E, T, V = precond.hl_to_gl_matrices(k)
    op = P.Operator(mesh, k, 2.0, "hermite_like", dtype)
    x = uniform_vector(op.ndofs, seed=20 + k)
    if dtype == "f32":
        x = x.astype(np.float32).astype(np.float64)
    tol = 1e-12 if dtype == "f64" else 1e-5
    for mode, M in (("T", T), ("TT", T.T), ("VALUES", E.T)):
        y = op.basis_change(mode, _dev(torch, x, dtype)).cpu().numpy().astype(np.float64)
        ref = precond.apply_cellwise(precond.kron3(M), x, ncells)
        e2, emax = rel_errors(y, ref)
        assert e2 <= tol and emax <= tol, (mode, e2, emax)
    op.close()


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 7])
@pytest.mark.parametrize("mesh_name", ["deformed", "affine"])
def test_gl_diagonal_and_pjacobi(k, mesh_name):
    """diag(A_GL) equals the diagonal of the oracle's GL matrix, and P^-1 of
    eq. (jacobi) equals the oracle's (T^T)^{x3} diag^-1 T^{x3}."""
    torch, P = require_gpu()
    banner(f"gl diagonal + pjacobi k={k} {mesh_name}")
    mesh = unit_cube((3, 2, 2), 0.1) if mesh_name == "deformed" else paper_affine_brick((2, 3, 2))
    Ag = SIPG(mesh, k, 2.0, "nodal_gl").assemble()
    dg = Ag.diagonal()
    op = P.Operator(mesh, k, 2.0, "hermite_like", "f64")
    d = op.compute_gl_diagonal().cpu().numpy()
    e2, emax = rel_errors(d, dg)
    assert e2 <= 1e-12 and emax <= 1e-12, (e2, emax)
    r = uniform_vector(op.ndofs, seed=5)
    z = op.basis_change("PJACOBI", _dev(torch, r, "f64")).cpu().numpy()
    ref = precond.pjacobi_hl(k, dg, r, mesh.ncells)
    e2, emax = rel_errors(z, ref)
    assert e2 <= 1e-12 and emax <= 1e-12, (e2, emax)
    op.close()


def test_gl_operator_diagonal_matches_own_basis():
    """For the nodal operator the GL diagonal is its own matrix diagonal."""
    torch, P = require_gpu()
    banner("gl diagonal of GL operator")
    mesh = unit_cube((2, 2, 3), 0.1)
    k = 3
    dg = SIPG(mesh, k, 2.0, "nodal_gl").assemble().diagonal()
    op = P.Operator(mesh, k, 2.0, "nodal_gl", "f64")
    d = op.compute_gl_diagonal().cpu().numpy()
    assert rel_errors(d, dg)[1] <= 1e-12
    op.close()


def test_pjacobi_requires_diagonal():
    torch, P = require_gpu()
    op = P.Operator(unit_cube(2), 2, 2.0)
    x = op.empty()
    with pytest.raises(P.SipgError):
        op.basis_change("PJACOBI", x)
    op.close()


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("mesh_name", ["brick", "deformed", "affine"])
@pytest.mark.parametrize("basis", ["hermite_like", "nodal_gl", "nodal_gauss"])
def test_fdm_block_preconditioner(k, mesh_name, basis):
    """SIPG_BC_FDM (fast diagonalization on the device) equals the oracle's
    explicit solve with the Kronecker-sum block of eq. (KDlaplace_dg)."""
    from oracle import fdm
    from workloads import Mesh
    torch, P = require_gpu()
    banner(f"fdm k={k} {mesh_name} {basis}")
    mesh = {"brick": Mesh(n=(3, 2, 4), lo=(0.0, -0.5, 0.0), hi=(0.75, 1.0, 0.8)),
            "deformed": unit_cube((2, 3, 2), 0.1),
            "affine": paper_affine_brick((2, 2, 3))}[mesh_name]
    r = uniform_vector(mesh.ncells * (k + 1) ** 3, seed=40 + k)
    ref = fdm.apply(mesh, k, 2.0, basis, r)
    for dtype, tol in (("f64", 1e-12), ("f32", 1e-5)):
        op = P.Operator(mesh, k, 2.0, basis, dtype)
        rr = r if dtype == "f64" else r.astype(np.float32).astype(np.float64)
        z = op.basis_change("FDM", _dev(torch, rr, dtype)).cpu().numpy().astype(np.float64)
        ref_d = ref if dtype == "f64" else fdm.apply(mesh, k, 2.0, basis, rr)
        e2, emax = rel_errors(z, ref_d)
        assert e2 <= tol and emax <= tol, (dtype, e2, emax)
        op.close()
