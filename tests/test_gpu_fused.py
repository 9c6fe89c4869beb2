"""GPU parity of the fused product and preconditioner (sipg_apply_pjacobi):
y = A x and z = P^-1 y of eq. (jacobi) in one pass.  Against the FP64 oracle
for the Hermite-like basis (the oracle's P^-1 is written for it), and against
the separate entry points (sipg_apply, then sipg_basis_change PJACOBI) for
every basis and precision.

Tolerances: as the separate paths' parity tests (FP64 1e-12 relative in the
2-norm and the max-norm; FP32 1e-5); y must equal sipg_apply's bit for bit."""
import numpy as np
import pytest

from oracle import precond
from oracle.sipg import SIPG
from workloads import paper_affine_brick, unit_cube, uniform_vector
from tests.gpu_util import banner, rel_errors, require_gpu

pytestmark = pytest.mark.gpu

# 14 cells: the last workgroup is partial for every n <= 6
ORACLE_MESHES = {
    "deformed": lambda: unit_cube((7, 2, 1), 0.1),
    "affine": lambda: paper_affine_brick((2, 7, 1)),
    "cartesian": lambda: unit_cube((1, 2, 7)),
}
# larger mesh for the checks against the separate entry points
DEFORMED = lambda: unit_cube((3, 4, 5), 0.1)  # noqa: E731


def _gl_diagonal_oracle(mesh, k):
    # diag(A_GL): the diagonal of each cell's own block of the nodal GL matrix
    akk, _ = SIPG(mesh, k, 2.0, "nodal_gl").local_blocks()
    return np.einsum("cii->ci", akk).reshape(-1)


def _fused(torch, P, mesh, k, basis, dtype, x):
    op = P.Operator(mesh, k, 2.0, basis, dtype)
    op.compute_gl_diagonal(return_diag=False)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    xd = torch.from_numpy(x).to("cuda", dtype=tdt)
    y, z = op.apply_pjacobi(xd)
    y_sep = op.apply(xd)
    z_sep = op.basis_change("PJACOBI", y_sep)
    torch.cuda.synchronize()
    out = [t.cpu().numpy() for t in (y, z, y_sep, z_sep)]
    op.close()
    return out


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("mesh_name", list(ORACLE_MESHES))
def test_apply_pjacobi_f64_against_oracle(mesh_name, k):
    torch, P = require_gpu()
    banner(f"apply_pjacobi f64 {mesh_name} k={k}")
    mesh = ORACLE_MESHES[mesh_name]()
    ref_op = SIPG(mesh, k, 2.0, "hermite_like")
    x = uniform_vector(ref_op.ndofs, seed=30 + k)
    y_ref = ref_op.apply_naive(x)
    z_ref = precond.pjacobi_hl(k, _gl_diagonal_oracle(mesh, k), y_ref, mesh.ncells)
    y, z, y_sep, z_sep = _fused(torch, P, mesh, k, "hermite_like", "f64", x)
    assert np.array_equal(y, y_sep)
    e2, emax = rel_errors(y, y_ref)
    assert e2 <= 1e-12 and emax <= 1e-12, (e2, emax)
    e2, emax = rel_errors(z, z_ref)
    assert e2 <= 1e-12 and emax <= 1e-12, (e2, emax)
    assert np.max(np.abs(z - z_sep)) <= 1e-14 * np.max(np.abs(z_sep))


@pytest.mark.parametrize("k", [6, 7, 8])
def test_apply_pjacobi_high_degree_matches_separate_calls(k):
    # both separate paths are checked against the oracle in their own tests
    torch, P = require_gpu()
    banner(f"apply_pjacobi f64 deformed k={k}")
    mesh = DEFORMED()
    x = uniform_vector(mesh.ncells * (k + 1) ** 3, seed=30 + k)
    y, z, y_sep, z_sep = _fused(torch, P, mesh, k, "hermite_like", "f64", x)
    assert np.array_equal(y, y_sep)
    assert np.max(np.abs(z - z_sep)) <= 1e-14 * np.max(np.abs(z_sep))


@pytest.mark.parametrize("k", [2, 4, 5])
def test_apply_pjacobi_f32_against_oracle(k):
    torch, P = require_gpu()
    banner(f"apply_pjacobi f32 deformed k={k}")
    mesh = ORACLE_MESHES["deformed"]()
    ref_op = SIPG(mesh, k, 2.0, "hermite_like")
    x = uniform_vector(ref_op.ndofs, seed=40 + k).astype(np.float32).astype(np.float64)
    y_ref = ref_op.apply_naive(x)
    z_ref = precond.pjacobi_hl(k, _gl_diagonal_oracle(mesh, k), y_ref, mesh.ncells)
    y, z, y_sep, z_sep = _fused(torch, P, mesh, k, "hermite_like", "f32", x)
    assert np.array_equal(y, y_sep)
    for got, ref in ((y, y_ref), (z, z_ref)):
        e2, emax = rel_errors(got.astype(np.float64), ref)
        assert e2 <= 1e-5 and emax <= 1e-5, (e2, emax)


@pytest.mark.parametrize("k", [2, 4, 7])
@pytest.mark.parametrize("basis", ["nodal_gl", "nodal_gauss"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_apply_pjacobi_other_bases_match_separate_calls(basis, k, dtype):
    torch, P = require_gpu()
    banner(f"apply_pjacobi {basis} k={k} {dtype}")
    mesh = DEFORMED()
    n3 = (k + 1) ** 3
    x = uniform_vector(mesh.ncells * n3, seed=50 + k)
    y, z, y_sep, z_sep = _fused(torch, P, mesh, k, basis, dtype, x)
    assert np.array_equal(y, y_sep)
    tol = 1e-14 if dtype == "f64" else 1e-6
    assert np.max(np.abs(z - z_sep)) <= tol * np.max(np.abs(z_sep))


def test_apply_pjacobi_argument_errors():
    torch, P = require_gpu()
    op = P.Operator(unit_cube(2), 2, 2.0)
    x = torch.zeros(op.ndofs, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SipgError):          # no GL diagonal yet
        op.apply_pjacobi(x)
    op.compute_gl_diagonal(return_diag=False)
    y = op.empty()
    with pytest.raises(P.SipgError):          # z overlaps y
        op.apply_pjacobi(x, y, y)
    with pytest.raises(P.SipgError):          # z overlaps x
        op.apply_pjacobi(x, y, x)
    op.close()
