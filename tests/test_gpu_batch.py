"""GPU tests of the batched product (sipg_batch_*): every output of a batch
of independent operators equals the single-operator product bit for bit
(same kernel body, same summation order) and the FP64 oracle to the stated
tolerance; overlapping outputs are rejected."""
import numpy as np
import pytest

from oracle.sipg import SIPG
from workloads import Mesh, paper_affine_brick, unit_cube, uniform_vector
from tests.gpu_util import banner, rel_errors, require_gpu

pytestmark = pytest.mark.gpu


def _mixed_specs(rng, count):
    """(mesh, k, basis, dtype) with ragged cell counts, degrees 1..8, both
    bases and precisions, affine and deformed meshes."""
    specs = []
    for i in range(count):
        n = tuple(int(v) for v in rng.integers(1, 5, size=3))
        kind = i % 3
        mesh = (unit_cube(n, 0.1) if kind == 0 else paper_affine_brick(n) if kind == 1
                else Mesh(n=n, lo=(0.0, -0.5, 0.25), hi=(1.0, 1.0, 1.0)))
        k = int(rng.integers(1, 9))
        basis = "hermite_like" if rng.random() < 0.7 else "nodal_gl"
        dtype = "f64" if rng.random() < 0.6 else "f32"
        specs.append((mesh, k, basis, dtype))
    return specs


def _setup(torch, P, specs, seed0=0):
    ops, xs, ys = [], [], []
    for i, (mesh, k, basis, dtype) in enumerate(specs):
        op = P.Operator(mesh, k, 2.0, basis, dtype)
        tdt = torch.float64 if dtype == "f64" else torch.float32
        x = uniform_vector(op.ndofs, seed0 + i)
        ops.append(op)
        xs.append(torch.from_numpy(x).to(device="cuda", dtype=tdt))
        ys.append(torch.full((op.ndofs,), float("nan"), dtype=tdt, device="cuda"))
    return ops, xs, ys


def test_batch_equals_single_products_and_oracle():
    torch, P = require_gpu()
    banner("batch mixed 40 operators")
    rng = np.random.default_rng(11)
    specs = _mixed_specs(rng, 40)
    ops, xs, ys = _setup(torch, P, specs)
    b = P.Batch(ops, xs, ys)
    keys = {(op.degree, op.basis, op.dtype_name, op.info.geometry, op.info.diagonal_metric) for op in ops}
    assert b.info.nops == 40 and b.info.launches == len(keys)
    assert b.info.ndofs == sum(op.ndofs for op in ops)
    b.apply()
    torch.cuda.synchronize()
    for i, (op, x, y) in enumerate(zip(ops, xs, ys)):
        single = op.apply(x)
        torch.cuda.synchronize()
        assert torch.equal(y, single), i
    # the oracle on a few of them (FP64 1e-12, FP32 1e-5 on the rounded input)
    for i in range(0, 40, 5):
        mesh, k, basis, dtype = specs[i]
        ref = SIPG(mesh, k, 2.0, basis).apply_naive(xs[i].double().cpu().numpy())
        e2, emax = rel_errors(ys[i].double().cpu().numpy(), ref)
        tol = 1e-12 if dtype == "f64" else 1e-5
        assert e2 <= tol and emax <= tol, (i, specs[i], e2, emax)
    b.close()
    for op in ops:
        op.close()


def test_batch_rebinds_by_pointer_and_shares_inputs():
    """The batch reads the bound buffers at each apply; several operators may
    read one input."""
    torch, P = require_gpu()
    banner("batch shared input")
    mesh = unit_cube((3, 2, 4), 0.1)
    ops = [P.Operator(mesh, 3, 2.0, "hermite_like", "f64") for _ in range(3)]
    ops.append(P.Operator(mesh, 3, 1.0, "hermite_like", "f64"))
    x = torch.from_numpy(uniform_vector(ops[0].ndofs, 5)).cuda()
    ys = [torch.empty_like(x) for _ in ops]
    b = P.Batch(ops, [x] * 4, ys)
    assert b.info.launches == 1
    b.apply()
    torch.cuda.synchronize()
    assert torch.equal(ys[0], ys[1]) and torch.equal(ys[0], ys[2])
    assert not torch.equal(ys[0], ys[3])     # other penalty factor
    x.copy_(torch.from_numpy(uniform_vector(ops[0].ndofs, 6)))
    b.apply()
    torch.cuda.synchronize()
    ref = SIPG(mesh, 3, 2.0).apply_naive(x.cpu().numpy())
    e2, emax = rel_errors(ys[1].cpu().numpy(), ref)
    assert e2 <= 1e-12 and emax <= 1e-12
    b.close()
    for op in ops:
        op.close()


def test_batch_rejects_overlapping_outputs():
    torch, P = require_gpu()
    banner("batch overlap errors")
    mesh = unit_cube(2)
    a = P.Operator(mesh, 2, 2.0)
    c = P.Operator(mesh, 2, 2.0)
    buf = torch.zeros(4 * a.ndofs, dtype=torch.float64, device="cuda")
    x0, x1, y0 = buf[:a.ndofs], buf[a.ndofs:2 * a.ndofs], buf[2 * a.ndofs:3 * a.ndofs]
    y_shift = buf[a.ndofs // 2:a.ndofs // 2 + a.ndofs]          # meets x0 and x1
    cases = [([a, c], [x0, x1], [y0, y0]),                         # two outputs alike
             ([a, c], [x0, x1], [y0, y_shift]),                    # output over inputs
             ([a], [x0], [x0])]                                    # in place
    for ops, xs, ys in cases:
        with pytest.raises(P.SipgError) as e:
            P.Batch(ops, xs, ys)
        assert e.value.code == -1 and "overlaps" in str(e.value)
    a.close()
    c.close()


def test_batch_many_small_operators_one_launch():
    """256 one-cell-to-64-cell operators of one degree: one grid, every result
    bit-identical to its own launch."""
    torch, P = require_gpu()
    banner("batch 256 small operators")
    rng = np.random.default_rng(3)
    ops, xs, ys = [], [], []
    for i in range(256):
        n = tuple(int(v) for v in rng.integers(1, 5, size=3))
        op = P.Operator(unit_cube(n, 0.1 if i % 2 else 0.0), 4, 2.0, "hermite_like", "f64", "qpoint")
        ops.append(op)
        xs.append(torch.from_numpy(uniform_vector(op.ndofs, 1000 + i)).cuda())
        ys.append(torch.empty_like(xs[-1]))
    b = P.Batch(ops, xs, ys)
    assert b.info.launches == 1
    b.apply()
    torch.cuda.synchronize()
    for op, x, y in zip(ops, xs, ys):
        assert torch.equal(y, op.apply(x))
    b.close()
    for op in ops:
        op.close()


def test_batch_tune_keeps_results():
    """The schedule autotuner may switch groups to one launch per operator;
    the outputs stay bit-identical."""
    torch, P = require_gpu()
    banner("batch tune")
    rng = np.random.default_rng(5)
    specs = _mixed_specs(rng, 16)
    ops, xs, ys = _setup(torch, P, specs, seed0=50)
    b = P.Batch(ops, xs, ys)
    b.apply()
    torch.cuda.synchronize()
    before = [y.clone() for y in ys]
    b.tune(2)
    assert 0 <= b.info.per_operator_groups <= b.info.launches
    for y in ys:
        y.fill_(float("nan"))
    b.apply()
    torch.cuda.synchronize()
    for y0, y1 in zip(before, ys):
        assert torch.equal(y0, y1)
    b.close()
    for op in ops:
        op.close()
