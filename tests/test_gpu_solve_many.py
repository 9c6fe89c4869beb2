"""Several right-hand sides of one multigrid solver solved together
(sipg_mg_solve_many: one iteration loop for all of them) against the same
solves one at a time, and their residuals against the oracle's operator."""
import numpy as np
import pytest

from oracle import mms
from oracle.sipg import SIPG
from workloads import unit_cube
from tests.gpu_util import banner, require_gpu

pytestmark = pytest.mark.gpu


def _rhs_rows(P, mesh, k, nrhs, seed):
    """Rows of differing difficulty: sums of sine modes, one zero row, one
    row scaled by 1e3 and one random vector."""
    torch, _ = require_gpu()
    op = P.Operator(mesh, k, 2.0)
    rng = np.random.default_rng(seed)
    rows = []
    for v in range(nrhs):
        if v == 1:
            rows.append(torch.zeros(op.ndofs, dtype=torch.float64, device="cuda"))
        elif v == 3:
            rows.append(torch.from_numpy(rng.uniform(-1, 1, op.ndofs)).cuda())
        else:
            amps = rng.normal(size=4) * (1e3 if v == 2 else 1.0)
            waves = rng.integers(1, 5, size=(4, 3))
            rows.append(op.assemble_rhs(list(amps), [tuple(w) for w in waves]))
    op.close()
    return torch.stack(rows).contiguous()


CASES = [
    # mesh, degree, precision, multigrid options
    ("cube6", 3, "mixed", {}),
    ("deformed6", 4, "f64", {"smoother": "pjacobi"}),
    ("cube7", 3, "mixed", {"p_coarsening": 1, "smoother": "fdm"}),
    ("deformed5", 5, "mixed", {"p_coarsening": 1, "coarse_direct_max_dofs": 256}),
    ("cube4", 2, "f64", {"fused_smoother": 0}),
    ("cube4x2x6", 6, "mixed", {"p_coarsening": 2}),
]
MESHES = {"cube6": unit_cube(6), "deformed6": unit_cube(6, 0.1), "cube7": unit_cube(7),
          "deformed5": unit_cube(5, 0.1), "cube4": unit_cube(4), "cube4x2x6": unit_cube((4, 2, 6))}


@pytest.mark.parametrize("name,k,precision,opts", CASES, ids=[c[0] + f"-k{c[1]}-{c[2]}" for c in CASES])
def test_solve_many_equals_one_by_one(name, k, precision, opts):
    torch, P = require_gpu()
    banner(f"solve_many {name} k={k} {precision} {opts}")
    mesh = MESHES[name]
    mg = P.Multigrid(mesh, k, 2.0, precision=precision, **opts)
    nrhs = 5
    b = _rhs_rows(P, mesh, k, nrhs, seed=k)
    tol = 1e-9
    x, infos = mg.solve_many(b, rel_tol=tol, max_iter=100)
    xs = x.cpu().numpy()
    for v in range(nrhs):
        # the same iterations on the same data: the same iterate
        x1, info1 = mg.solve(b[v].contiguous(), rel_tol=tol, max_iter=100)
        x1 = x1.cpu().numpy()
        assert infos[v].iterations == info1.iterations, (v, infos[v], info1)
        scale = max(np.max(np.abs(x1)), 1e-300)
        assert np.max(np.abs(xs[v] - x1)) <= 1e-13 * scale, (v, np.max(np.abs(xs[v] - x1)) / scale)
        assert abs(infos[v].final_residual - info1.final_residual) <= 1e-12 * max(info1.final_residual, 1e-300)
        bn = float(torch.linalg.norm(b[v]))
        assert infos[v].true_residual <= 1.01 * tol * max(bn, 1.0), (v, infos[v], bn)
    # the zero right-hand side needs no iteration and keeps x = 0
    assert infos[1].iterations == 0 and not np.any(xs[1])
    mg.close()


def test_solve_many_single_rhs_and_initial_guess():
    """nrhs = 1 is sipg_mg_solve; a non-zero initial guess is used."""
    torch, P = require_gpu()
    banner("solve_many nrhs=1, initial guess")
    mesh = unit_cube(4, 0.1)
    k = 3
    mg = P.Multigrid(mesh, k, 2.0, precision="mixed")
    b = _rhs_rows(P, mesh, k, 3, seed=7)
    x0 = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, b.shape)).cuda()
    x, infos = mg.solve_many(b[:1].contiguous(), x0[:1].clone(), rel_tol=1e-10)
    x1, info1 = mg.solve(b[0].contiguous(), x0[0].clone(), rel_tol=1e-10)
    assert infos[0].iterations == info1.iterations
    assert torch.equal(x[0], x1)
    xm, im = mg.solve_many(b, x0.clone(), rel_tol=1e-10)
    for v in range(3):
        xv, iv = mg.solve(b[v].contiguous(), x0[v].clone(), rel_tol=1e-10)
        assert im[v].iterations == iv.iterations
        assert float(torch.max(torch.abs(xm[v] - xv))) <= 1e-13 * float(torch.max(torch.abs(xv)))
    mg.close()


def test_solve_many_residual_against_oracle():
    """The solutions of 16 right-hand sides (the maximum) meet the tolerance
    with the oracle's assembled operator."""
    torch, P = require_gpu()
    banner("solve_many 16 rhs vs oracle residual")
    mesh = unit_cube((3, 4, 2), 0.1)
    k = 3
    ref = SIPG(mesh, k, 2.0)
    A = ref.assemble()
    mg = P.Multigrid(mesh, k, 2.0, precision="mixed")
    rng = np.random.default_rng(11)
    B = rng.uniform(-1, 1, (16, ref.ndofs))
    x, infos = mg.solve_many(torch.from_numpy(B).cuda(), rel_tol=1e-10)
    X = x.cpu().numpy()
    for v in range(16):
        r = np.linalg.norm(B[v] - A @ X[v]) / np.linalg.norm(B[v])
        assert r <= 2e-10, (v, r)
        assert infos[v].iterations > 0
    mg.close()


def test_solve_many_sine_source_matches_oracle_solution():
    """A served request's source solved among others equals the oracle's
    direct solve of the same system."""
    torch, P = require_gpu()
    banner("solve_many sine source vs oracle direct solve")
    import scipy.sparse.linalg as spla
    mesh = unit_cube(3)
    k = 4
    ref = SIPG(mesh, k, 2.0)
    amps, waves = [1.0, -0.5], [(1, 2, 1), (3, 1, 2)]
    b_ref = mms.rhs(ref, mms.modes_rhs(amps, waves))
    x_ref = spla.spsolve(ref.assemble().tocsc(), b_ref)
    op = P.Operator(mesh, k, 2.0)
    b0 = op.assemble_rhs(amps, waves)
    op.close()
    b = torch.stack([b0, 2.0 * b0, -b0]).contiguous()
    mg = P.Multigrid(mesh, k, 2.0, precision="mixed")
    x, infos = mg.solve_many(b, rel_tol=1e-12)
    X = x.cpu().numpy()
    for v, s in enumerate((1.0, 2.0, -1.0)):
        e = np.linalg.norm(X[v] - s * x_ref) / np.linalg.norm(s * x_ref)
        assert e <= 1e-9, (v, e)
    mg.close()


def test_solve_many_noconv_and_arguments():
    torch, P = require_gpu()
    banner("solve_many max_iter and argument errors")
    mesh = unit_cube(4, 0.1)
    k = 3
    mg = P.Multigrid(mesh, k, 2.0, precision="mixed")
    b = _rhs_rows(P, mesh, k, 4, seed=5)
    x, infos = mg.solve_many(b, rel_tol=1e-14, max_iter=2, raise_on_noconv=False)
    assert all(i.status == P.SIPG_E_NOCONV for i in infos)
    assert infos[1].iterations == 0
    assert all(i.iterations == 2 for j, i in enumerate(infos) if j != 1)
    # the first two iterations are those of the one-by-one solves
    for v in (0, 2):
        xv, iv = mg.solve(b[v].contiguous(), rel_tol=1e-14, max_iter=2, raise_on_noconv=False)
        assert float(torch.max(torch.abs(x[v] - xv))) <= 1e-13 * float(torch.max(torch.abs(xv)))
    with pytest.raises(P.SipgError):
        mg.solve_many(torch.zeros((17, mg.ndofs), dtype=torch.float64, device="cuda"))
    with pytest.raises(P.SipgError):
        mg.solve_many(b, b)   # x overlapping b
    with pytest.raises(ValueError):
        mg.solve_many(b[:, :-1].contiguous())
    mg.close()
