"""The allocation-free CG entry point (sipg_cg_solve_static), called through
the C ABI, against sipg_cg_solve on the same operators: two calls in a row,
the second with a smaller operator, then an operator above the fixed
capacity (rejected before any device work)."""
import ctypes as C

import numpy as np
import pytest

from tests.gpu_util import banner, require_gpu
from workloads import unit_cube

pytestmark = pytest.mark.gpu


def _solve(P, fn, op, b, x, tol, maxit, stream):
    info = P.SipgSolveInfo()
    rc = fn(op.handle, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), C.c_double(tol), C.c_int(maxit),
            C.byref(info), C.c_void_p(stream))
    return rc, info


def test_cg_solve_static_matches_cg_solve():
    torch, P = require_gpu()
    assert P.lib.sipg_cg_static_max_dofs() == 1 << 20
    stream = int(torch.cuda.current_stream().cuda_stream)
    # larger first, then smaller: the second call finds the first one's data
    # in the fixed arrays and must not depend on it
    for mesh, k in ((unit_cube((8, 8, 8), 0.1), 3), (unit_cube((3, 4, 2)), 2)):
        banner(f"cg static vs allocating: {mesh.n} k={k}")
        op = P.Operator(mesh, k, 2.0, "hermite_like", "f64")
        b = op.assemble_rhs([3 * np.pi ** 2, 1.5], [(1, 1, 1), (2, 1, 3)])
        x_ref = torch.zeros_like(b)
        x_st = torch.zeros_like(b)
        rc1, i1 = _solve(P, P.lib.sipg_cg_solve, op, b, x_ref, 1e-10, 2000, stream)
        rc2, i2 = _solve(P, P.lib.sipg_cg_solve_static, op, b, x_st, 1e-10, 2000, stream)
        torch.cuda.synchronize()
        assert rc1 == 0 and rc2 == 0, (rc1, rc2, P.lib.sipg_last_error())
        assert i1.iterations == i2.iterations > 0
        # same kernels in the same order on the same data: bit-identical
        assert torch.equal(x_ref, x_st)
        assert i1.true_residual == i2.true_residual
        assert i2.true_residual <= 1.5e-10 * float(torch.linalg.norm(b))
        op.close()


def test_cg_solve_static_rejects_large_operator():
    torch, P = require_gpu()
    banner("cg static capacity")
    op = P.Operator(unit_cube(32), 3, 2.0)      # 2,097,152 unknowns > 2^20
    b = torch.ones(op.ndofs, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    rc, _ = _solve(P, P.lib.sipg_cg_solve_static, op, b, x, 1e-10, 10,
                   int(torch.cuda.current_stream().cuda_stream))
    assert rc == P.SIPG_E_ARG
    assert "fixed work arrays" in P.lib.sipg_last_error().decode()
    torch.cuda.synchronize()
    assert float(x.abs().max()) == 0.0          # nothing ran
    op.close()
