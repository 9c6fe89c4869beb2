"""GPU parity: the HIP matrix-free product against the FP64 CPU oracle.

Tolerances: FP64 relative 1e-12 (2-norm and max-norm), FP32 relative 1e-5
against the FP64 oracle applied to the float32-rounded input."""
import numpy as np
import pytest

from oracle.sipg import SIPG
from workloads import PAPER_BRICK_HI, PAPER_BRICK_LO, PAPER_LINEAR_MAP, Mesh, paper_affine_brick, unit_cube, uniform_vector
from tests.gpu_util import banner, rel_errors, require_gpu

pytestmark = pytest.mark.gpu

MESHES = {
    # cell counts chosen so that the last workgroup is partial for every n
    "cartesian": unit_cube((5, 3, 4)),
    "deformed": unit_cube((3, 4, 5), 0.1),
    "paper_affine": paper_affine_brick((4, 3, 2)),
    "brick_aniso": Mesh(n=(2, 5, 3), lo=(0.0, -1.0, 0.5), hi=(1.0, 1.5, 1.1)),
    # graded bricks (sipg_mesh.width: the last cell of each direction narrower),
    # the coarse levels of meshes with odd cell counts
    "graded": Mesh(n=(3, 4, 2), width=(0.4, 0.3, 0.6)),
    "graded_deformed": Mesh(n=(4, 3, 3), width=(0.3, 0.4, 0.4), deform_amp=0.1),
    "graded_affine": Mesh(n=(3, 2, 2), lo=PAPER_BRICK_LO, hi=PAPER_BRICK_HI, lin=PAPER_LINEAR_MAP,
                          width=(0.7, 1.0, 0.9)),
}
_oracle_cache = {}


def oracle(mesh_name, k, basis, eta=2.0):
    key = (mesh_name, k, basis, eta)
    if key not in _oracle_cache:
        _oracle_cache[key] = SIPG(MESHES[mesh_name], k, eta, basis)
    return _oracle_cache[key]


def run_apply(torch, P, mesh, k, basis, dtype, x, geometry="auto", eta=2.0):
    op = P.Operator(mesh, k, eta, basis, dtype, geometry)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    xd = torch.from_numpy(x).to(device="cuda", dtype=tdt)
    y = op.apply(xd)
    torch.cuda.synchronize()
    out = y.cpu().numpy().astype(np.float64)
    op.close()
    return out


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("basis", ["hermite_like", "nodal_gl", "nodal_gauss"])
@pytest.mark.parametrize("mesh_name", list(MESHES))
def test_apply_f64(mesh_name, basis, k):
    torch, P = require_gpu()
    banner(f"apply f64 {mesh_name} {basis} k={k}")
    ref_op = oracle(mesh_name, k, basis)
    x = uniform_vector(ref_op.ndofs, seed=k)
    ref = ref_op.apply_naive(x)
    y = run_apply(torch, P, MESHES[mesh_name], k, basis, "f64", x)
    e2, emax = rel_errors(y, ref)
    assert e2 <= 1e-12 and emax <= 1e-12, (e2, emax)


@pytest.mark.parametrize("k", [2, 4, 7])
@pytest.mark.parametrize("mesh_name", ["paper_affine", "cartesian"])
def test_apply_f64_per_point_geometry_on_affine_mesh(mesh_name, k):
    """The per-quadrature-point metric path on an affine mesh gives the same operator."""
    torch, P = require_gpu()
    banner(f"apply f64 qpoint {mesh_name} k={k}")
    ref_op = oracle(mesh_name, k, "hermite_like")
    x = uniform_vector(ref_op.ndofs, seed=100 + k)
    y = run_apply(torch, P, MESHES[mesh_name], k, "hermite_like", "f64", x, geometry="qpoint")
    e2, emax = rel_errors(y, ref_op.apply_naive(x))
    assert e2 <= 1e-12 and emax <= 1e-12, (e2, emax)


@pytest.mark.parametrize("geometry,mesh_name,expected", [
    ("auto", "cartesian", 1), ("auto", "brick_aniso", 1), ("auto", "paper_affine", 0),
    ("auto", "deformed", 0), ("qpoint", "cartesian", 0), ("cell", "brick_aniso", 1), ("auto", "graded", 1),
    ("auto", "graded_affine", 0)])
def test_diagonal_metric_variant(geometry, mesh_name, expected):
    """Per-cell storage of an affine map with a diagonal linear part selects the
    reference-coordinate cell term (sipg_op_info.diagonal_metric); the other
    operators keep the quadrature cell term.  Both are checked against the
    oracle by the parity tests above."""
    torch, P = require_gpu()
    banner(f"diagonal metric {geometry} {mesh_name}")
    op = P.Operator(MESHES[mesh_name], 3, 2.0, "hermite_like", "f64", geometry)
    assert op.info.diagonal_metric == expected
    op.close()


@pytest.mark.parametrize("k", [1, 3, 4, 5, 7, 8])
@pytest.mark.parametrize("basis", ["hermite_like", "nodal_gl", "nodal_gauss"])
@pytest.mark.parametrize("mesh_name", ["deformed", "paper_affine", "cartesian", "graded_deformed"])
def test_apply_f32(mesh_name, basis, k):
    torch, P = require_gpu()
    banner(f"apply f32 {mesh_name} {basis} k={k}")
    ref_op = oracle(mesh_name, k, basis)
    x = uniform_vector(ref_op.ndofs, seed=k).astype(np.float32)
    ref = ref_op.apply_naive(x.astype(np.float64))
    y = run_apply(torch, P, MESHES[mesh_name], k, basis, "f32", x)
    e2, emax = rel_errors(y, ref)
    assert e2 <= 1e-5 and emax <= 1e-5, (e2, emax)


def test_small_config_against_assembled_matrix():
    """8^3 Cartesian unit cube, k=3, eta=2, x ~ U[-1,1] seed 0: y = A x with A
    assembled explicitly by the oracle."""
    torch, P = require_gpu()
    banner("small config 8^3 k=3 vs CSR")
    mesh = unit_cube(8)
    ref_op = SIPG(mesh, 3, 2.0)
    A = ref_op.assemble()
    x = uniform_vector(ref_op.ndofs, seed=0)
    y = run_apply(torch, P, mesh, 3, "hermite_like", "f64", x)
    e2, emax = rel_errors(y, A @ x)
    assert e2 <= 1e-12 and emax <= 1e-12, (e2, emax)


@pytest.mark.parametrize("k", [2, 5])
@pytest.mark.parametrize("eta", [1.0, 3.5])
def test_penalty_factor(k, eta):
    torch, P = require_gpu()
    banner(f"penalty eta={eta} k={k}")
    mesh = MESHES["deformed"]
    ref_op = SIPG(mesh, k, eta)
    x = uniform_vector(ref_op.ndofs, seed=7)
    y = run_apply(torch, P, mesh, k, "hermite_like", "f64", x, eta=eta)
    e2, emax = rel_errors(y, ref_op.apply_naive(x))
    assert e2 <= 1e-12 and emax <= 1e-12, (e2, emax)


@pytest.mark.parametrize("n", [(1, 1, 1), (1, 1, 7), (7, 1, 1), (1, 6, 1), (2, 1, 1)])
def test_degenerate_meshes(n):
    """Single cells and single-cell-thick slabs: every face is a boundary face
    in some direction."""
    torch, P = require_gpu()
    banner(f"degenerate mesh {n}")
    for k in (1, 4):
        mesh = unit_cube(n, 0.1)
        ref_op = SIPG(mesh, k, 2.0)
        x = uniform_vector(ref_op.ndofs, seed=3)
        y = run_apply(torch, P, mesh, k, "hermite_like", "f64", x)
        e2, emax = rel_errors(y, ref_op.apply_naive(x))
        assert e2 <= 1e-12 and emax <= 1e-12, (k, e2, emax)


def test_hermite_like_reads_only_two_neighbour_layers():
    """Section 4.2: changing a neighbour's unknowns outside its value and
    derivative layers leaves y of the cell bit-identical."""
    torch, P = require_gpu()
    banner("two-layer access")
    k, n = 4, 5
    mesh = unit_cube((3, 3, 3), 0.1)
    x = uniform_vector(mesh.ncells * n ** 3, seed=11)
    y0 = run_apply(torch, P, mesh, k, "hermite_like", "f64", x)
    centre = 13                                        # cell (1,1,1)
    X = x.reshape(27, n, n, n).copy()                  # [cell, i3, i2, i1]
    for nb, axis, layers in ((12, 3, (n - 1, n - 2)), (14, 3, (0, 1)), (10, 2, (n - 1, n - 2)),
                             (16, 2, (0, 1)), (4, 1, (n - 1, n - 2)), (22, 1, (0, 1))):
        keep = np.zeros(n, bool)
        keep[list(layers)] = True
        sl = [slice(None)] * 3
        sl[axis - 1] = ~keep
        blk = X[nb]
        blk[tuple(sl)] += 0.37
    y1 = run_apply(torch, P, mesh, k, "hermite_like", "f64", X.reshape(-1))
    Y0 = y0.reshape(27, -1)
    Y1 = y1.reshape(27, -1)
    assert np.array_equal(Y0[centre], Y1[centre])
    assert not np.array_equal(Y0[12], Y1[12])


@pytest.mark.parametrize("k,basis,dtype", [(4, "hermite_like", "f64"), (2, "nodal_gl", "f64"), (3, "hermite_like", "f32")])
def test_z_interleaved_block_order(k, basis, dtype):
    # 50 z-layers: the kernel's XCD ranges hold full groups of three
    # interleaved z-layers of blocks and a shorter last group in plain order
    torch, P = require_gpu()
    banner(f"z-interleaved block order {basis} k={k} {dtype}")
    mesh = unit_cube((4, 3, 50), 0.1)
    ref_op = SIPG(mesh, k, 2.0, basis)
    x = uniform_vector(ref_op.ndofs, seed=11)
    if dtype == "f32":
        x = x.astype(np.float32).astype(np.float64)
    ref = ref_op.apply_naive(x)
    y = run_apply(torch, P, mesh, k, basis, dtype, x)
    e2, emax = rel_errors(y, ref)
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert e2 <= tol and emax <= tol, (e2, emax)


def test_deterministic():
    torch, P = require_gpu()
    banner("determinism")
    mesh = unit_cube((6, 5, 4), 0.1)
    op = P.Operator(mesh, 5, 2.0)
    x = torch.from_numpy(uniform_vector(op.ndofs, 5)).cuda()
    a = op.apply(x).cpu().numpy()
    b = op.apply(x).cpu().numpy()
    assert np.array_equal(a, b)
    op.close()
