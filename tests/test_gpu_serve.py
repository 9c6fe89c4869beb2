"""GPU tests of the request loop (sipg_submit / sipg_poll): every result is
the same alone and in the mix, within the stated tolerance, and the memory
budget admits, evicts or rejects requests as documented."""
import numpy as np
import pytest

from tests.gpu_util import banner, require_gpu
from workloads import unit_cube

pytestmark = pytest.mark.gpu


def _requests(rng, count):
    out = []
    for _ in range(count):
        n = int(rng.integers(3, 9))
        k = int(rng.integers(2, 5))
        amps = rng.normal(size=4)
        waves = rng.integers(1, 4, size=(4, 3))
        out.append((n, k, amps, waves))
    return out


def test_single_request_matches_direct_solve():
    torch, P = require_gpu()
    banner("serve single request")
    mesh = unit_cube(6)
    amps, waves = [3 * np.pi ** 2], [(1, 1, 1)]
    srv = P.Server(workers=2, precision="mixed")
    t = srv.submit(P.Server.make_request(mesh, 3, amps, waves, rel_tol=1e-10))
    res = srv.wait(t)
    assert res["status"] == 0 and res["rel_residual"] <= 1.5e-10
    x = srv.solution(res)
    # the same problem solved directly with the multigrid solver
    op = P.Operator(mesh, 3, 2.0)
    b = op.assemble_rhs(amps, waves)
    mg = P.Multigrid(mesh, 3, 2.0, precision="mixed", smoother="fdm", p_coarsening=1,
                     coarse_reduction=10.0, graded_coarsening=0,
                     coarse_direct_max_dofs=256)   # the server's defaults
    xd, info = mg.solve(b, rel_tol=1e-10)
    torch.cuda.synchronize()
    assert info.iterations == res["iterations"]
    assert torch.equal(x, xd)          # same kernels, same order: bit-identical
    srv.release(t)
    srv.close()
    mg.close()
    op.close()


def test_results_same_alone_and_in_the_mix():
    torch, P = require_gpu()
    banner("serve mix")
    rng = np.random.default_rng(7)
    reqs = _requests(rng, 24)
    # alone: one worker, one request at a time
    alone = []
    srv = P.Server(workers=1, precision="mixed")
    for n, k, amps, waves in reqs:
        t = srv.submit(P.Server.make_request(unit_cube(n), k, amps, waves, rel_tol=1e-8))
        r = srv.wait(t)
        alone.append((r, srv.solution(r).cpu()))
        srv.release(t)
    srv.close()
    # in the mix: all submitted at once, four concurrent workers
    srv = P.Server(workers=4, precision="mixed")
    tickets = [srv.submit(P.Server.make_request(unit_cube(n), k, amps, waves, rel_tol=1e-8))
               for n, k, amps, waves in reqs]
    pending = set(tickets)
    polls = 0
    while pending:
        for t in list(pending):
            if srv.poll(t) is not None:
                pending.discard(t)
        polls += 1
    for t, (ra, xa) in zip(tickets, alone):
        rm = srv.wait(t)
        assert rm["status"] == 0 and rm["rel_residual"] <= 1e-8
        xm = srv.solution(rm).cpu()
        assert rm["iterations"] == ra["iterations"]
        rel = float((xm - xa).norm() / xa.norm())
        assert rel <= 1e-12, rel
        srv.release(t)
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["queued"] == 0
    srv.close()


def test_poll_not_ready_then_done():
    torch, P = require_gpu()
    banner("serve poll")
    srv = P.Server(workers=1)
    t = srv.submit(P.Server.make_request(unit_cube(16, 0.1), 4, [1.0], [(1, 2, 1)], rel_tol=1e-9))
    first = srv.poll(t)
    res = srv.wait(t)
    assert first is None or first["status"] == 0
    assert res["status"] == 0 and res["total_s"] >= res["solve_s"] > 0
    srv.release(t)
    srv.close()


def test_budget_rejects_and_evicts():
    torch, P = require_gpu()
    banner("serve budget")
    srv = P.Server(hbm_budget_bytes=64 << 20, workers=2)
    with pytest.raises(P.SipgError) as e:
        srv.submit(P.Server.make_request(unit_cube(40), 5, [1.0], [(1, 1, 1)]))
    assert e.value.code == -7
    # several distinct small problems: the cache must evict to stay in budget
    tickets = [srv.submit(P.Server.make_request(unit_cube(n), 3, [1.0], [(1, 1, 1)], rel_tol=1e-8))
               for n in (6, 8, 10, 6, 8, 10)]
    for t in tickets:
        r = srv.wait(t)
        assert r["status"] == 0 and r["rel_residual"] <= 1e-8
        srv.release(t)
    st = srv.stats()
    assert st["peak_bytes"] <= 64 << 20
    srv.close()


def test_server_with_block_jacobi_smoother_matches_direct_solve():
    torch, P = require_gpu()
    banner("serve fdm smoother")
    mesh = unit_cube(8, 0.1)
    amps, waves = [1.0, -0.5], [(1, 1, 1), (2, 3, 1)]
    srv = P.Server(workers=2, precision="mixed", smoother="fdm")
    t = srv.submit(P.Server.make_request(mesh, 4, amps, waves, rel_tol=1e-9))
    res = srv.wait(t)
    assert res["status"] == 0 and res["rel_residual"] <= 1e-9
    op = P.Operator(mesh, 4, 2.0)
    b = op.assemble_rhs(amps, waves)
    mg = P.Multigrid(mesh, 4, 2.0, precision="mixed", smoother="fdm", p_coarsening=1, coarse_reduction=10.0,
                     graded_coarsening=0, coarse_direct_max_dofs=256)
    xd, info = mg.solve(b, rel_tol=1e-9)
    torch.cuda.synchronize()
    assert info.iterations == res["iterations"]
    assert torch.equal(srv.solution(res), xd)
    srv.release(t)
    srv.close()
    mg.close()
    op.close()


def test_server_with_graded_levels_matches_direct_solve():
    """The server's graded coarsening option (odd meshes coarsened through
    graded bricks down to a dense coarse solve) gives the direct solve's
    result, bit for bit."""
    torch, P = require_gpu()
    banner("serve graded levels")
    mesh = unit_cube(9)
    amps, waves = [1.0, 0.3], [(1, 1, 1), (1, 2, 3)]
    srv = P.Server(workers=2, precision="mixed", graded_coarsening=1, coarse_direct_max_dofs=256)
    t = srv.submit(P.Server.make_request(mesh, 3, amps, waves, rel_tol=1e-9))
    res = srv.wait(t)
    assert res["status"] == 0 and res["rel_residual"] <= 1e-9
    op = P.Operator(mesh, 3, 2.0)
    b = op.assemble_rhs(amps, waves)
    mg = P.Multigrid(mesh, 3, 2.0, precision="mixed", smoother="fdm", p_coarsening=1, coarse_reduction=10.0,
                     graded_coarsening=1, coarse_direct_max_dofs=256)
    assert mg.info.coarse_steps == 0 and mg.info.levels >= 4
    xd, info = mg.solve(b, rel_tol=1e-9)
    torch.cuda.synchronize()
    assert info.iterations == res["iterations"]
    assert torch.equal(srv.solution(res), xd)
    srv.release(t)
    srv.close()
    mg.close()
    op.close()


def test_server_solves_queued_requests_of_one_problem_together():
    """Requests of one problem queued behind a running solve are taken along
    into one multi-right-hand-side solve (sipg_mg_solve_many); every result
    is its own direct solve's, bit for bit, and other problems in between
    are served as before."""
    torch, P = require_gpu()
    banner("serve grouped requests")
    rng = np.random.default_rng(21)
    mesh, k = unit_cube(6), 3
    other, ko = unit_cube(5, 0.1), 2
    specs = []
    # the queued requests of each problem sit at scattered places of a queue
    # with many others behind them: taking them out must leave exactly the rest
    for i in range(16):
        m, d = (mesh, k) if i in (0, 1, 2, 4, 9, 15) else (other, ko)
        specs.append((m, d, list(rng.normal(size=3)), [tuple(w) for w in rng.integers(1, 4, size=(3, 3))]))
    # one worker: while it builds the first hierarchy the rest queue up
    srv = P.Server(workers=1, precision="mixed", batch_max_rhs=8)
    tickets = [srv.submit(P.Server.make_request(m, d, a, w, rel_tol=1e-9)) for m, d, a, w in specs]
    results = [srv.wait(t) for t in tickets]
    st = srv.stats()
    assert st["batched_solves"] >= 2 and st["batched_requests"] >= 4, st
    assert st["completed"] == len(specs) and st["queued"] == 0, st
    mgs = {}
    for (m, d, a, w), t, res in zip(specs, tickets, results):
        assert res["status"] == 0 and res["rel_residual"] <= 1e-9, res
        if d not in mgs:
            mgs[d] = (P.Operator(m, d, 2.0),
                      P.Multigrid(m, d, 2.0, precision="mixed", smoother="fdm", p_coarsening=1,
                                  coarse_reduction=10.0, graded_coarsening=0, coarse_direct_max_dofs=256))
        op, mg = mgs[d]
        xd, info = mg.solve(op.assemble_rhs(a, w), rel_tol=1e-9)
        torch.cuda.synchronize()
        assert info.iterations == res["iterations"], (info, res)
        assert torch.equal(srv.solution(res), xd)
        srv.release(t)
    srv.close()
    for op, mg in mgs.values():
        mg.close()
        op.close()
    # batching off: every request alone
    srv = P.Server(workers=1, precision="mixed", batch_max_rhs=1)
    tickets = [srv.submit(P.Server.make_request(m, d, a, w, rel_tol=1e-9)) for m, d, a, w in specs[:4]]
    for t in tickets:
        assert srv.wait(t)["status"] == 0
        srv.release(t)
    assert srv.stats()["batched_solves"] == 0
    srv.close()
