"""Device memory through the caller's allocator (sipg_allocator): with
PyTorch's caching allocator the operator, the CG workspace, the multigrid
hierarchy and served results come from torch's pool and go back to it."""
import numpy as np
import pytest

from tests.gpu_util import banner, require_gpu
from workloads import unit_cube

pytestmark = pytest.mark.gpu


def _rounded(nbytes):
    # torch's caching allocator rounds each block up to a multiple of 512 bytes
    return 512 * ((nbytes + 511) // 512)


def test_operator_memory_comes_from_torch():
    torch, P = require_gpu()
    banner("allocator: operator")
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    op = P.Operator(unit_cube((6, 5, 4), 0.1), 3, 2.0)
    m1 = torch.cuda.memory_allocated()
    # tables, cell metric, block-preconditioner scalars, 3 face arrays
    assert op.info.device_bytes <= m1 - m0 <= op.info.device_bytes + 6 * 512
    op.compute_gl_diagonal(return_diag=False)
    m2 = torch.cuda.memory_allocated()
    assert m2 - m1 == _rounded(8 * op.ndofs)
    # the CG workspace is taken and returned within the call
    b = op.assemble_rhs([1.0], [(1, 1, 1)])
    m3 = torch.cuda.memory_allocated()
    x, info = op.cg_solve(b, rel_tol=1e-8)
    assert torch.cuda.memory_allocated() == m3 + _rounded(8 * op.ndofs)   # only x
    del x, b
    op.close()
    assert torch.cuda.memory_allocated() == m0


def test_operator_with_hip_malloc_leaves_torch_pool_alone():
    torch, P = require_gpu()
    banner("allocator: hipMalloc")
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    op = P.Operator(unit_cube(4, 0.1), 2, 2.0, allocator=None)
    assert torch.cuda.memory_allocated() == m0
    op.close()


def test_multigrid_memory_comes_from_torch():
    torch, P = require_gpu()
    banner("allocator: multigrid")
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    mg = P.Multigrid(unit_cube(8), 3, 2.0, precision="mixed")
    m1 = torch.cuda.memory_allocated()
    assert m1 - m0 >= 0.9 * mg.info.device_bytes
    b = torch.ones(mg.ndofs, dtype=torch.float64, device="cuda")
    x, info = mg.solve(b, rel_tol=1e-8)
    assert info.status == 0
    del x, b
    mg.close()
    assert torch.cuda.memory_allocated() == m0


def test_release_waits_for_callers_copy():
    """A solution copied on a side stream and released right away (on that
    stream) is copied whole: the buffer is freed only after the copy."""
    torch, P = require_gpu()
    banner("serve release after copy")
    srv = P.Server(workers=2, precision="mixed")
    mesh = unit_cube(8)
    amps, waves = [3 * np.pi ** 2], [(1, 1, 1)]
    t = srv.submit(P.Server.make_request(mesh, 3, amps, waves, rel_tol=1e-10))
    res = srv.wait(t)
    ref = srv.solution(res).cpu()
    t2 = srv.submit(P.Server.make_request(mesh, 3, amps, waves, rel_tol=1e-10))
    res2 = srv.wait(t2)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        sol = srv.solution(res2, stream=side)
        srv.release(t2, stream=side)
        # whatever reuses the freed block comes after the copy
        junk = torch.full((int(res2["ndofs"]),), 7.0, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    assert torch.equal(sol.cpu(), ref)
    del junk
    srv.release(t)
    srv.close()
