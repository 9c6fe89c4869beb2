"""GPU parity of the right-hand side, the multigrid transfer and the
multigrid-preconditioned solves against the oracle."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import mms
from oracle import multigrid as omg
from oracle.sipg import SIPG
from workloads import Mesh, unit_cube, paper_affine_brick
from tests.gpu_util import banner, rel_errors, require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k", [1, 3, 5, 8])
@pytest.mark.parametrize("deform", [0.0, 0.1])
def test_rhs_sines(k, deform):
    torch, P = require_gpu()
    banner(f"rhs k={k} deform={deform}")
    mesh = unit_cube((3, 2, 4), deform)
    ref = SIPG(mesh, k, 2.0)
    amps = [3 * np.pi ** 2, -0.7, 1.3]
    waves = [(1, 1, 1), (2, 1, 3), (4, 2, 1)]
    b_ref = mms.rhs(ref, mms.modes_rhs(amps, waves))
    op = P.Operator(mesh, k, 2.0)
    b = op.assemble_rhs(amps, waves).cpu().numpy()
    e2, emax = rel_errors(b, b_ref)
    assert e2 <= 1e-12 and emax <= 1e-12, (e2, emax)
    op.close()


@pytest.mark.parametrize("k", [1, 2, 4, 7])
@pytest.mark.parametrize("basis", ["hermite_like", "nodal_gl", "nodal_gauss"])
def test_transfer_matches_oracle(k, basis):
    torch, P = require_gpu()
    banner(f"transfer k={k} {basis}")
    mesh = unit_cube((4, 2, 6), 0.1)
    mg = P.Multigrid(mesh, k, 2.0, basis, precision="f64", lanczos_steps=4)
    nf, cf = mg.level(0)
    nc, cc = mg.level(1)
    assert cf == (4, 2, 6) and cc == (2, 1, 3)
    rng = np.random.default_rng(k)
    c = rng.uniform(-1, 1, nc)
    f = rng.uniform(-1, 1, nf)
    dc = torch.from_numpy(c).cuda()
    df = torch.from_numpy(f).cuda()
    out_f = torch.empty(nf, dtype=torch.float64, device="cuda")
    out_c = torch.empty(nc, dtype=torch.float64, device="cuda")
    pf = mg.transfer(0, "prolongate", dc, out_f).cpu().numpy()
    rc = mg.transfer(0, "restrict", df, out_c).cpu().numpy()
    e = rel_errors(pf, omg.prolongate(c, cf, basis, k))
    assert e[0] < 1e-12 and e[1] < 1e-12, e
    e = rel_errors(rc, omg.restrict(f, cf, basis, k))
    assert e[0] < 1e-12 and e[1] < 1e-12, e
    mg.close()


def test_vcycle_is_symmetric_in_fp64():
    """The V-cycle (Chebyshev pre/post smoothing, transposed transfers) is a
    symmetric operator, as CG requires."""
    torch, P = require_gpu()
    banner("vcycle symmetry")
    mesh = unit_cube((4, 4, 4), 0.1)
    mg = P.Multigrid(mesh, 3, 2.0, precision="f64")
    rng = np.random.default_rng(2)
    a = torch.from_numpy(rng.uniform(-1, 1, mg.ndofs)).cuda()
    b = torch.from_numpy(rng.uniform(-1, 1, mg.ndofs)).cuda()
    va = mg.vcycle(a)
    vb = mg.vcycle(b)
    lhs = float(torch.dot(b, va))
    rhs = float(torch.dot(a, vb))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs), (lhs, rhs)
    assert float(torch.dot(a, va)) > 0
    mg.close()


@pytest.mark.parametrize("precision", ["mixed", "f64"])
def test_mg_solve_small_config(precision):
    """8^3 Cartesian unit cube, k=3, eta=2, manufactured sine solution:
    residual 1e-10 in FP64 and the same discrete solution as the oracle."""
    torch, P = require_gpu()
    banner(f"mg solve small {precision}")
    mesh = unit_cube(8)
    ref = SIPG(mesh, 3, 2.0)
    A = ref.assemble()
    b = mms.rhs(ref, mms.sine_rhs)
    mg = P.Multigrid(mesh, 3, 2.0, precision=precision)
    assert mg.info.levels == 4
    x, info = mg.solve(torch.from_numpy(b).cuda(), rel_tol=1e-10)
    xs = x.cpu().numpy()
    res = np.linalg.norm(b - A @ xs) / np.linalg.norm(b)
    assert res <= 1.5e-10, res
    assert info.iterations <= 20, info.iterations
    xr, _ = spla.cg(A, b, rtol=1e-13, maxiter=20000)
    assert rel_errors(xs, xr)[0] < 1e-8
    mg.close()


@pytest.mark.parametrize("precision", ["mixed", "f64"])
def test_mg_solve_deformed_k5(precision):
    torch, P = require_gpu()
    banner(f"mg solve deformed k=5 {precision}")
    mesh = unit_cube(6, 0.1)
    ref = SIPG(mesh, 5, 2.0)
    b = mms.rhs(ref, mms.sine_rhs)
    mg = P.Multigrid(mesh, 5, 2.0, precision=precision)
    x, info = mg.solve(torch.from_numpy(b).cuda(), rel_tol=1e-10)
    xs = x.cpu().numpy()
    r = b - ref.apply_naive(xs)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.5e-10
    assert info.iterations <= 25, info.iterations
    assert mms.l2_error(ref, xs, mms.sine) < 1e-4
    mg.close()


def test_mg_solve_gl_basis_and_affine_brick():
    torch, P = require_gpu()
    banner("mg solve GL basis, paper brick")
    mesh = paper_affine_brick((4, 4, 2))
    ref = SIPG(mesh, 4, 2.0, "nodal_gl")
    rng = np.random.default_rng(0)
    b = rng.uniform(-1, 1, ref.ndofs)
    mg = P.Multigrid(mesh, 4, 2.0, "nodal_gl", precision="mixed")
    x, info = mg.solve(torch.from_numpy(b).cuda(), rel_tol=1e-10)
    r = b - ref.apply_naive(x.cpu().numpy())
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.5e-10
    mg.close()


@pytest.mark.parametrize("precision", ["mixed", "f64"])
@pytest.mark.parametrize("case", ["cartesian_k3", "deformed_k5", "affine_k4_gl"])
def test_mg_solve_with_block_jacobi_smoother(precision, case):
    """Chebyshev smoothing around the block-Jacobi preconditioner of Section
    6.4 converges to the same discrete solution.  On the Cartesian mesh, where
    the block is the exact interior cell matrix, it needs no more iterations
    than point Jacobi (Table 5); on the deformed and affine meshes the block is
    the axis-aligned approximation and only convergence is required."""
    torch, P = require_gpu()
    banner(f"mg solve fdm {case} {precision}")
    mesh, k, basis = {"cartesian_k3": (unit_cube(8), 3, "hermite_like"),
                      "deformed_k5": (unit_cube(6, 0.1), 5, "hermite_like"),
                      "affine_k4_gl": (paper_affine_brick((4, 4, 2)), 4, "nodal_gl")}[case]
    ref = SIPG(mesh, k, 2.0, basis)
    b = mms.rhs(ref, mms.sine_rhs)
    its = {}
    for sm in ("pjacobi", "fdm"):
        mg = P.Multigrid(mesh, k, 2.0, basis, precision=precision, smoother=sm)
        x, info = mg.solve(torch.from_numpy(b).cuda(), rel_tol=1e-10)
        xs = x.cpu().numpy()
        r = b - ref.apply_naive(xs)
        assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.5e-10, sm
        its[sm] = info.iterations
        mg.close()
    if case == "cartesian_k3":
        assert its["fdm"] <= its["pjacobi"], its


def test_vcycle_with_block_jacobi_is_symmetric_in_fp64():
    torch, P = require_gpu()
    banner("vcycle symmetry fdm")
    mesh = unit_cube((4, 4, 4), 0.1)
    mg = P.Multigrid(mesh, 3, 2.0, precision="f64", smoother="fdm")
    rng = np.random.default_rng(4)
    a = torch.from_numpy(rng.uniform(-1, 1, mg.ndofs)).cuda()
    b = torch.from_numpy(rng.uniform(-1, 1, mg.ndofs)).cuda()
    lhs = float(torch.dot(b, mg.vcycle(a)))
    rhs = float(torch.dot(a, mg.vcycle(b)))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs), (lhs, rhs)
    mg.close()


@pytest.mark.parametrize("rule,degrees", [(1, [5, 2, 1]), (2, [4, 3, 2, 1])])
@pytest.mark.parametrize("basis", ["hermite_like", "nodal_gl"])
def test_degree_transfer_matches_oracle(rule, degrees, basis):
    """Levels that lower the degree on an odd mesh (no mesh coarsening is
    possible): prolongation and restriction between degrees equal the oracle's
    embedding and its transpose."""
    torch, P = require_gpu()
    banner(f"degree transfer rule={rule} {basis}")
    mesh = unit_cube((3, 2, 3), 0.1)
    mg = P.Multigrid(mesh, degrees[0], 2.0, basis, precision="f64", lanczos_steps=4, p_coarsening=rule)
    assert mg.info.levels == len(degrees)
    assert [mg.level_degree(l) for l in range(len(degrees))] == degrees
    rng = np.random.default_rng(rule)
    for l in range(len(degrees) - 1):
        kf, kc = degrees[l], degrees[l + 1]
        nf, _ = mg.level(l)
        nc, cells = mg.level(l + 1)
        assert cells == (3, 2, 3)
        c = rng.uniform(-1, 1, nc)
        f = rng.uniform(-1, 1, nf)
        out_f = torch.empty(nf, dtype=torch.float64, device="cuda")
        out_c = torch.empty(nc, dtype=torch.float64, device="cuda")
        pf = mg.transfer(l, "prolongate", torch.from_numpy(c).cuda(), out_f).cpu().numpy()
        rc = mg.transfer(l, "restrict", torch.from_numpy(f).cuda(), out_c).cpu().numpy()
        e = rel_errors(pf, omg.p_prolongate(c, mesh.ncells, basis, kf, kc))
        assert e[0] < 1e-12 and e[1] < 1e-12, (l, e)
        e = rel_errors(rc, omg.p_restrict(f, mesh.ncells, basis, kf, kc))
        assert e[0] < 1e-12 and e[1] < 1e-12, (l, e)
    mg.close()


def test_degree_then_mesh_levels():
    """p levels first, then mesh coarsening at the lowest degree; the mesh
    transfer of that level matches the oracle at degree 1."""
    torch, P = require_gpu()
    banner("p then h levels")
    mesh = unit_cube((4, 2, 6), 0.1)
    mg = P.Multigrid(mesh, 3, 2.0, precision="f64", lanczos_steps=4, p_coarsening=1)
    assert [mg.level_degree(l) for l in range(mg.info.levels)] == [3, 1, 1]
    assert mg.level(2)[1] == (2, 1, 3)
    nc, _ = mg.level(2)
    c = np.random.default_rng(9).uniform(-1, 1, nc)
    nf, _ = mg.level(1)
    out_f = torch.empty(nf, dtype=torch.float64, device="cuda")
    pf = mg.transfer(1, "prolongate", torch.from_numpy(c).cuda(), out_f).cpu().numpy()
    e = rel_errors(pf, omg.prolongate(c, (4, 2, 6), "hermite_like", 1))
    assert e[0] < 1e-12 and e[1] < 1e-12, e
    mg.close()


@pytest.mark.parametrize("precision", ["mixed", "f64"])
@pytest.mark.parametrize("rule", [1, 2])
def test_mg_solve_odd_mesh_with_degree_levels(precision, rule):
    """7^3 cells (odd: no mesh coarsening) with degree levels converges to
    1e-10 in few iterations and gives the oracle's discrete solution."""
    torch, P = require_gpu()
    banner(f"mg solve odd mesh rule={rule} {precision}")
    mesh = unit_cube(7, 0.1)
    ref = SIPG(mesh, 4, 2.0)
    b = mms.rhs(ref, mms.sine_rhs)
    mg = P.Multigrid(mesh, 4, 2.0, precision=precision, p_coarsening=rule)
    x, info = mg.solve(torch.from_numpy(b).cuda(), rel_tol=1e-10)
    xs = x.cpu().numpy()
    r = b - ref.apply_naive(xs)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.5e-10
    assert info.iterations <= 25, info.iterations
    assert mg.info.coarse_steps < 400, mg.info.coarse_steps
    mg.close()


def test_vcycle_with_degree_levels_is_symmetric_in_fp64():
    torch, P = require_gpu()
    banner("vcycle symmetry p levels")
    mesh = unit_cube((4, 4, 2), 0.1)
    mg = P.Multigrid(mesh, 5, 2.0, precision="f64", p_coarsening=1)
    rng = np.random.default_rng(6)
    a = torch.from_numpy(rng.uniform(-1, 1, mg.ndofs)).cuda()
    b = torch.from_numpy(rng.uniform(-1, 1, mg.ndofs)).cuda()
    lhs = float(torch.dot(b, mg.vcycle(a)))
    rhs = float(torch.dot(a, mg.vcycle(b)))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs), (lhs, rhs)
    mg.close()


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("mesh_name", ["affine", "deformed"])
@pytest.mark.parametrize("rule", [0, 1])
@pytest.mark.parametrize("smoother", ["pjacobi", "fdm"])
def test_fused_smoother_matches_two_launch_degrees(k, mesh_name, rule, smoother):
    """The fused Chebyshev step against the two-launch smoother for every
    degree: n = 3..9 (wavefront-local and block-barrier cell steps, early and
    late metric loads), per-cell (unit cube: diagonal metric) and per-point
    (deformed) geometry, with and without degree levels; one V-cycle in FP64
    and in mixed precision, and equal CG iteration counts."""
    torch, P = require_gpu()
    banner(f"fused smoother k={k} {mesh_name} p_coarsening={rule} {smoother}")
    mesh = unit_cube((4, 2, 2), 0.1 if mesh_name == "deformed" else 0.0)
    r = np.random.default_rng(90 + k).uniform(-1, 1, mesh.ncells * (k + 1) ** 3)
    for precision in ("f64", "mixed"):
        out, its = [], []
        for fused in (1, 0):
            mg = P.Multigrid(mesh, k, 2.0, precision=precision, smoother=smoother, fused_smoother=fused,
                             p_coarsening=rule, lanczos_steps=8)
            out.append(mg.vcycle(torch.from_numpy(r).cuda()).cpu().numpy())
            x, info = mg.solve(torch.from_numpy(r).cuda(), rel_tol=1e-9, max_iter=100)
            its.append(info.iterations)
            mg.close()
        diff = np.max(np.abs(out[0] - out[1])) / np.max(np.abs(out[1]))
        assert diff <= (1e-13 if precision == "f64" else 1e-6), (precision, diff)
        assert its[0] == its[1], (precision, its)


@pytest.mark.parametrize("k", [3, 5])
@pytest.mark.parametrize("mesh_name", ["cartesian", "deformed"])
def test_hermite_like_with_gl_basis_change_equals_gl_point_jacobi(k, mesh_name):
    """Section 6.3: multigrid with the Hermite-like basis and point Jacobi in
    the nodal Gauss-Lobatto basis (through the basis change of eq. (jacobi))
    is the same method as multigrid in the Gauss-Lobatto basis with point
    Jacobi.  With A_GL = V^T A_HL V and P_HL^-1 = V diag(A_GL)^-1 V^T the
    smoothed operators are similar, the coarse spaces are the same, and with
    the same eigenvalue-estimate start in both bases (lanczos_start = 1) the
    two preconditioned CG runs produce x_HL = V x_GL iterate by iterate."""
    torch, P = require_gpu()
    banner(f"HL+GL basis change vs GL point Jacobi k={k} {mesh_name}")
    mesh = unit_cube(4, 0.1 if mesh_name == "deformed" else 0.0)
    amps, waves = [3 * np.pi ** 2, 0.8], [(1, 1, 1), (2, 3, 1)]
    res = {}
    for basis in ("hermite_like", "nodal_gl"):
        op = P.Operator(mesh, k, 2.0, basis)
        b = op.assemble_rhs(amps, waves)
        mg = P.Multigrid(mesh, k, 2.0, basis, precision="f64", smoother="pjacobi", lanczos_start=1)
        # a fixed number of iterations (the residual norms differ by V^T)
        x6, info6 = mg.solve(b, rel_tol=1e-30, max_iter=6, raise_on_noconv=False)
        x, info = mg.solve(b, rel_tol=1e-10)
        res[basis] = (x6, x, info.iterations, mg.info.lambda_max_fine, op)
        mg.close()
    hl, gl = res["hermite_like"], res["nodal_gl"]
    # the same eigenvalue estimate (similar operators, equivalent starts)
    assert abs(hl[3] - gl[3]) <= 1e-10 * gl[3], (hl[3], gl[3])
    # x_HL = V x_GL (V = T^T cell by cell: GL coefficients -> HL coefficients)
    for a, g in ((hl[0], gl[0]), (hl[1], gl[1])):
        mapped = hl[4].basis_change("TT", g)
        e = float(torch.linalg.norm(a - mapped) / torch.linalg.norm(a))
        assert e <= 1e-10, e
    assert hl[2] == gl[2], (hl[2], gl[2])
    hl[4].close()
    gl[4].close()


@pytest.mark.parametrize("smoother", ["pjacobi", "fdm"])
@pytest.mark.parametrize("precision", ["mixed", "f64"])
def test_fused_smoother_matches_two_launch_smoother(smoother, precision):
    """The Chebyshev step fused into the product (residual, P^-1 and update
    in the product's workgroups) gives the V-cycle of the product followed by
    the merged pass, up to rounding."""
    torch, P = require_gpu()
    banner(f"fused smoother {smoother} {precision}")
    mesh = unit_cube((4, 4, 6), 0.1)
    k = 4
    r = np.random.default_rng(9).uniform(-1, 1, mesh.ncells * (k + 1) ** 3)
    out = []
    for fused in (1, 0):
        mg = P.Multigrid(mesh, k, 2.0, precision=precision, smoother=smoother, fused_smoother=fused)
        assert mg.info.levels >= 2 and mg.ndofs == r.size
        out.append(mg.vcycle(torch.from_numpy(r).cuda()).cpu().numpy())
        x, info = mg.solve(torch.from_numpy(r).cuda(), rel_tol=1e-10)
        assert info.iterations <= 25
        mg.close()
    diff = np.max(np.abs(out[0] - out[1])) / np.max(np.abs(out[1]))
    assert diff <= (1e-13 if precision == "f64" else 1e-6), diff


# graded coarsening of a 5 x 4 x 3 unit cube (fine cells paired from 0 on, the
# last one alone for odd counts): one-child cells, then unequal pairs
GRADED_CHAIN = [unit_cube((5, 4, 3)),
                Mesh(n=(3, 2, 2), width=(0.4, 0.5, 2 / 3)),
                Mesh(n=(2, 1, 1), width=(0.8, 1.0, 4 / 3)),
                Mesh(n=(1, 1, 1), width=(1.6, 1.0, 4 / 3))]


@pytest.mark.parametrize("k", [1, 2, 5])
@pytest.mark.parametrize("basis", ["hermite_like", "nodal_gl", "nodal_gauss"])
def test_graded_transfer_matches_oracle(k, basis):
    """graded_coarsening: the level bricks are the expected graded bricks and
    every mesh transfer equals the oracle's embedding between the two nested
    bricks (found from the cell bounds alone)."""
    torch, P = require_gpu()
    banner(f"graded transfer k={k} {basis}")
    mg = P.Multigrid(GRADED_CHAIN[0], k, 2.0, basis, precision="f64", lanczos_steps=4, graded_coarsening=1)
    assert [mg.level(l)[1] for l in range(mg.info.levels)] == [m.n for m in GRADED_CHAIN]
    rng = np.random.default_rng(k)
    for l in range(3):
        fine, coarse = GRADED_CHAIN[l], GRADED_CHAIN[l + 1]
        nf, nc = mg.level(l)[0], mg.level(l + 1)[0]
        c = rng.uniform(-1, 1, nc)
        f = rng.uniform(-1, 1, nf)
        out_f = torch.empty(nf, dtype=torch.float64, device="cuda")
        out_c = torch.empty(nc, dtype=torch.float64, device="cuda")
        pf = mg.transfer(l, "prolongate", torch.from_numpy(c).cuda(), out_f).cpu().numpy()
        rc = mg.transfer(l, "restrict", torch.from_numpy(f).cuda(), out_c).cpu().numpy()
        e = rel_errors(pf, omg.prolongate_nested(c, fine, coarse, basis, k))
        assert e[0] < 1e-12 and e[1] < 1e-12, (l, e)
        e = rel_errors(rc, omg.restrict_nested(f, fine, coarse, basis, k))
        assert e[0] < 1e-12 and e[1] < 1e-12, (l, e)
    mg.close()


@pytest.mark.parametrize("precision", ["mixed", "f64"])
@pytest.mark.parametrize("k,mesh_name", [(1, "cube2"), (2, "brick")])
def test_direct_coarse_solve_is_exact(precision, k, mesh_name):
    """A level of at most coarse_direct_max_dofs unknowns is solved by its
    dense inverse: with one level the V-cycle is A^-1 (oracle: dense solve of
    the assembled matrix), and CG converges at once."""
    torch, P = require_gpu()
    banner(f"direct coarse {precision} k={k} {mesh_name}")
    mesh = unit_cube(2) if mesh_name == "cube2" else Mesh(n=(2, 1, 3), width=(0.6, 1.0, 0.4), deform_amp=0.1)
    ref = SIPG(mesh, k, 2.0)
    mg = P.Multigrid(mesh, k, 2.0, precision=precision, coarse_direct_max_dofs=ref.ndofs)
    assert mg.info.levels == 1 and mg.info.coarse_steps == 0
    r = np.random.default_rng(k).uniform(-1, 1, ref.ndofs)
    z = mg.vcycle(torch.from_numpy(r).cuda()).cpu().numpy()
    zref = np.linalg.solve(ref.assemble().toarray(), r)
    e = rel_errors(z, zref)
    tol = 1e-12 if precision == "f64" else 2e-5
    assert e[0] < tol, e
    # converged after the first iteration; the lagged stopping test may add one
    x, info = mg.solve(torch.from_numpy(r).cuda(), rel_tol=1e-10)
    assert info.iterations <= (2 if precision == "f64" else 4), info.iterations
    mg.close()


@pytest.mark.parametrize("precision", ["mixed", "f64"])
@pytest.mark.parametrize("n,k,deform", [(7, 4, 0.1), (9, 3, 0.0), (5, 5, 0.0)])
def test_mg_solve_graded_levels_with_direct_coarse(precision, n, k, deform):
    """Odd meshes coarsened by graded levels down to a dense coarse solve
    converge to 1e-10 and give the oracle's discrete solution."""
    torch, P = require_gpu()
    banner(f"mg solve graded n={n} k={k} {precision}")
    mesh = unit_cube(n, deform)
    ref = SIPG(mesh, k, 2.0)
    b = mms.rhs(ref, mms.sine_rhs)
    mg = P.Multigrid(mesh, k, 2.0, precision=precision, smoother="fdm", p_coarsening=1, coarse_reduction=10.0,
                     graded_coarsening=1, coarse_direct_max_dofs=256)
    assert mg.info.coarse_steps == 0
    cells = [mg.level(l)[1] for l in range(mg.info.levels)]
    assert cells[-1][0] < n and mg.level(mg.info.levels - 1)[0] <= 256, cells
    x, info = mg.solve(torch.from_numpy(b).cuda(), rel_tol=1e-10)
    r = b - ref.apply_naive(x.cpu().numpy())
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.5e-10
    assert info.iterations <= 25, info.iterations
    mg.close()
