"""GPU conjugate gradient solve (FP64) on the small configuration: 8^3
Cartesian unit cube, k=3, eta=2, manufactured u = sin(pi x) sin(pi y) sin(pi z),
relative residual 1e-10."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import mms
from oracle.sipg import SIPG
from workloads import unit_cube
from tests.gpu_util import banner, rel_errors, require_gpu

pytestmark = pytest.mark.gpu


def test_cg_small_config_mms():
    torch, P = require_gpu()
    banner("cg 8^3 k=3 mms")
    mesh = unit_cube(8)
    ref = SIPG(mesh, 3, 2.0)
    A = ref.assemble()
    b = mms.rhs(ref, mms.sine_rhs)
    op = P.Operator(mesh, 3, 2.0)
    bd = torch.from_numpy(b).cuda()
    x, info = op.cg_solve(bd, rel_tol=1e-10, max_iter=5000)
    xs = x.cpu().numpy()
    # the residual is checked with the oracle's assembled matrix
    res = np.linalg.norm(b - A @ xs) / np.linalg.norm(b)
    assert res <= 1.5e-10, res
    assert info.true_residual / np.linalg.norm(b) <= 1.5e-10
    # same discrete solution as an oracle solve to the same accuracy
    xr, _ = spla.cg(A, b, rtol=1e-13, maxiter=20000)
    assert rel_errors(xs, xr)[0] < 1e-7
    # and the discretization error of the paper's setting (order k+1)
    err = mms.l2_error(ref, xs, mms.sine)
    assert err < 2e-4, err
    op.close()


def test_cg_zero_rhs_and_noconv():
    torch, P = require_gpu()
    banner("cg edge cases")
    op = P.Operator(unit_cube(3), 2, 2.0)
    b = torch.zeros(op.ndofs, dtype=torch.float64, device="cuda")
    x, info = op.cg_solve(b, rel_tol=1e-10)
    assert info.iterations == 0 and float(x.abs().max()) == 0.0
    b = torch.ones(op.ndofs, dtype=torch.float64, device="cuda")
    x, info = op.cg_solve(b, rel_tol=1e-14, max_iter=3, raise_on_noconv=False)
    assert info.status == -6 and info.iterations == 3
    op.close()


def test_cg_without_caller_allocator_matches():
    """With no caller allocator the CG workspace is stream-ordered device
    memory; the solve is the same, bit for bit, and repeated calls work."""
    torch, P = require_gpu()
    banner("cg stream-ordered workspace")
    mesh = unit_cube((4, 3, 5), 0.1)
    b = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, 4 * 3 * 5 * 27)).cuda()
    a = P.Operator(mesh, 2, 2.0)
    n = P.Operator(mesh, 2, 2.0, allocator=None)
    xa, ia = a.cg_solve(b, rel_tol=1e-10)
    for _ in range(2):
        xn, i_n = n.cg_solve(b, rel_tol=1e-10)
        torch.cuda.synchronize()
        assert i_n.iterations == ia.iterations
        assert torch.equal(xn, xa)
    a.close()
    n.close()
