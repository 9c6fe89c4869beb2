"""One GPU's share of a z-slab partition: slab operators whose boundary faces
read the neighbours' layers from packed ghost buffers reproduce the rows of
the whole mesh's operator (and the oracle's)."""
import numpy as np
import pytest

from oracle.sipg import SIPG
from workloads import Mesh, paper_affine_brick, unit_cube, uniform_vector
from tests.gpu_util import banner, rel_errors, require_gpu

pytestmark = pytest.mark.gpu

CASES = {
    "deformed": (unit_cube((5, 4, 7), 0.1), [(0, 2), (2, 5), (5, 7)]),
    "paper_affine": (paper_affine_brick((3, 4, 6)), [(0, 3), (3, 6)]),
    "cartesian_thin": (unit_cube((4, 3, 5)), [(0, 1), (1, 2), (2, 5)]),
    # graded brick: the narrower last cell of z lies in the top slab
    "graded_deformed": (Mesh(n=(3, 4, 5), width=(0.4, 0.3, 0.22), deform_amp=0.1), [(0, 2), (2, 5)]),
}


def _slab_products(torch, P, mesh, k, basis, dtype, splits, x, pjacobi=False):
    n3 = (k + 1) ** 3
    per = mesh.n[0] * mesh.n[1] * n3
    ops = [P.Operator(mesh, k, 2.0, basis, dtype, slab=s) for s in splits]
    xs = [x[z0 * per:z1 * per].contiguous() for z0, z1 in splits]
    ys, zs = [], []
    for i, (op, xi) in enumerate(zip(ops, xs)):
        lo = ops[i - 1].pack_ghost(1, xs[i - 1]) if i > 0 else None
        hi = ops[i + 1].pack_ghost(0, xs[i + 1]) if i + 1 < len(ops) else None
        if pjacobi:
            op.compute_gl_diagonal(return_diag=False)
            y, z = op.apply_slab(xi, lo, hi, z=op.empty())
            zs.append(z)
        else:
            y = op.apply_slab(xi, lo, hi)
        ys.append(y)
    torch.cuda.synchronize()
    out = torch.cat(ys), (torch.cat(zs) if pjacobi else None)
    for op in ops:
        op.close()
    return out


@pytest.mark.parametrize("k", [1, 3, 4, 7])
@pytest.mark.parametrize("basis", ["hermite_like", "nodal_gl", "nodal_gauss"])
@pytest.mark.parametrize("case", list(CASES))
def test_slabs_reproduce_the_whole_operator(case, basis, k):
    torch, P = require_gpu()
    banner(f"slab {case} {basis} k={k}")
    mesh, splits = CASES[case]
    whole = P.Operator(mesh, k, 2.0, basis, "f64")
    x = torch.from_numpy(uniform_vector(whole.ndofs, k)).cuda()
    y_ref = whole.apply(x)
    y, _ = _slab_products(torch, P, mesh, k, basis, "f64", splits, x)
    scale = float(y_ref.abs().max())
    assert float((y - y_ref).abs().max()) <= 1e-14 * scale
    # and the oracle's rows of the middle slab
    z0, z1 = splits[1]
    cells = np.arange(z0 * mesh.n[0] * mesh.n[1], z1 * mesh.n[0] * mesh.n[1])
    ref = SIPG(mesh, k, 2.0, basis, cells=cells).apply_naive(x.cpu().numpy())
    per = mesh.n[0] * mesh.n[1] * (k + 1) ** 3
    e2, emax = rel_errors(y[z0 * per:z1 * per].cpu().numpy(), ref)
    assert e2 <= 1e-12 and emax <= 1e-12, (e2, emax)
    whole.close()


@pytest.mark.parametrize("basis", ["nodal_gl", "nodal_gauss"])
def test_slabs_fp32_nodal(basis):
    torch, P = require_gpu()
    banner(f"slab f32 {basis}")
    mesh, splits = CASES["deformed"]
    whole = P.Operator(mesh, 3, 2.0, basis, "f32")
    x = torch.from_numpy(uniform_vector(whole.ndofs, 9)).to("cuda", torch.float32)
    y_ref = whole.apply(x)
    y, _ = _slab_products(torch, P, mesh, 3, basis, "f32", splits, x)
    assert float((y - y_ref).abs().max()) <= 1e-6 * float(y_ref.abs().max())
    whole.close()


@pytest.mark.parametrize("k", [2, 4])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_slab_step_with_pjacobi(dtype, k):
    """The fused step (y and z = P^-1 y) on slabs equals the whole mesh's;
    the GL diagonal of a slab treats its boundary planes as interior faces."""
    torch, P = require_gpu()
    banner(f"slab step {dtype} k={k}")
    mesh, splits = CASES["deformed"]
    tdt = torch.float64 if dtype == "f64" else torch.float32
    whole = P.Operator(mesh, k, 2.0, "hermite_like", dtype)
    whole.compute_gl_diagonal(return_diag=False)
    x = torch.from_numpy(uniform_vector(whole.ndofs, 5)).to("cuda", tdt)
    y_ref, z_ref = whole.apply_pjacobi(x)
    y, z = _slab_products(torch, P, mesh, k, "hermite_like", dtype, splits, x, pjacobi=True)
    tol = 1e-14 if dtype == "f64" else 1e-6
    assert float((y - y_ref).abs().max()) <= tol * float(y_ref.abs().max())
    assert float((z - z_ref).abs().max()) <= tol * float(z_ref.abs().max())
    whole.close()


def test_slab_arguments():
    torch, P = require_gpu()
    banner("slab arguments")
    mesh = unit_cube((3, 3, 4), 0.1)
    mid = P.Operator(mesh, 2, 2.0, slab=(1, 3))
    bottom = P.Operator(mesh, 2, 2.0, slab=(0, 1))
    x = torch.zeros(mid.ndofs, dtype=torch.float64, device="cuda")
    g = mid.pack_ghost(0, x)
    assert g.numel() == 3 * 3 * 2 * 9 == mid.ghost_size()
    with pytest.raises(P.SipgError):
        mid.apply(x)                       # neighbours on both sides: ghosts required
    with pytest.raises(P.SipgError):
        mid.apply_slab(x, g, None)         # the upper ghost is missing
    xb = torch.zeros(bottom.ndofs, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SipgError):
        bottom.apply_slab(xb, g, g)        # no slab below the bottom one
    bottom.apply_slab(xb, None, g)
    torch.cuda.synchronize()
    mid.close()
    bottom.close()
