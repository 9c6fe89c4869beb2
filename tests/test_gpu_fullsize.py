"""Parity at the full benchmark sizes, in the launch configuration bench.py
times: the product (and the preconditioners) on the whole mesh, checked
against the FP64 oracle on sampled cells (corners, faces, edges and random
interior cells), whose rows the oracle computes one by one.

Tolerance: FP64 relative 1e-12 of the sampled rows' max-norm (the same bar
as the small cases); FP32 1e-5 against the oracle on the float32-rounded
input."""
import numpy as np
import pytest

from oracle import fdm
from oracle import precond
from oracle.sipg import SIPG
from workloads import CONFIGS, uniform_vector, with_basis
from tests.gpu_util import banner, require_gpu

pytestmark = pytest.mark.gpu


def _sample_cells(mesh, count, seed):
    nx, ny, nz = mesh.n
    corners = [ix + nx * (iy + ny * iz) for ix in (0, nx - 1) for iy in (0, ny - 1) for iz in (0, nz - 1)]
    faces = [nx // 2 + nx * (ny // 2 + ny * 0), 0 + nx * (ny // 2 + ny * (nz // 2)),
             nx - 1 + nx * (ny // 2 + ny * (nz // 2)), nx // 2 + nx * (ny - 1 + ny * (nz // 2))]
    rng = np.random.default_rng(seed)
    inner = rng.choice(mesh.ncells, count, replace=False).tolist()
    return np.unique(np.array(corners + faces + inner, dtype=np.int64))


def _rows(y, cells, n3):
    return np.asarray(y).reshape(-1, n3)[cells].reshape(-1)


CASES = [("scale_k4_64c_deformed", "hermite_like", "f64"),
         ("scale_k4_64c_affine", "hermite_like", "f64"),
         ("scale_k4_64c_deformed", "nodal_gl", "f64"),
         ("scale_k7_32c_deformed", "hermite_like", "f64"),
         ("scale_k7_32c_affine", "nodal_gauss", "f64"),
         ("mixed_k5_48c_deformed", "hermite_like", "f32"),
         ("scale_k4_64c_deformed", "hermite_like", "f32")]


@pytest.mark.parametrize("name,basis,dtype", CASES)
def test_full_size_matvec_on_sampled_cells(name, basis, dtype):
    torch, P = require_gpu()
    banner(f"full size {name} {basis} {dtype}")
    cfg = with_basis(CONFIGS[name], basis)
    mesh, k = cfg.mesh, cfg.degree
    n3 = (k + 1) ** 3
    op = P.Operator(mesh, k, cfg.eta, basis, dtype)
    x = uniform_vector(op.ndofs, 0)
    if dtype == "f32":
        x = x.astype(np.float32).astype(np.float64)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    xd = torch.from_numpy(x).to("cuda", dtype=tdt)
    y = op.apply(xd)
    torch.cuda.synchronize()
    cells = _sample_cells(mesh, 24, 1)
    y_s = _rows(y.cpu().numpy().astype(np.float64), cells, n3)
    del y, xd
    op.close()
    torch.cuda.empty_cache()
    ref = SIPG(mesh, k, cfg.eta, basis, cells=cells).apply_naive(x)
    tol = 1e-12 if dtype == "f64" else 1e-5
    err = np.max(np.abs(y_s - ref)) / np.max(np.abs(ref))
    assert err <= tol, err


@pytest.mark.parametrize("mode", ["PJACOBI", "FDM"])
def test_full_size_preconditioners_on_sampled_cells(mode):
    """P^-1 of eq. (jacobi) (GL point Jacobi) and the block Jacobi of Section
    6.4 on the headline mesh; both act cell by cell, so sampled cells are
    checked exactly."""
    torch, P = require_gpu()
    banner(f"full size {mode}")
    cfg = CONFIGS["scale_k4_64c_deformed"]
    mesh, k = cfg.mesh, cfg.degree
    n3 = (k + 1) ** 3
    op = P.Operator(mesh, k, cfg.eta)
    if mode == "PJACOBI":
        op.compute_gl_diagonal(return_diag=False)
    r = uniform_vector(op.ndofs, 3)
    z = op.basis_change(mode, torch.from_numpy(r).cuda())
    torch.cuda.synchronize()
    cells = _sample_cells(mesh, 24, 2)
    z_s = _rows(z.cpu().numpy(), cells, n3)
    del z
    op.close()
    torch.cuda.empty_cache()
    r_s = _rows(r, cells, n3)
    if mode == "PJACOBI":
        akk, _ = SIPG(mesh, k, cfg.eta, "nodal_gl", cells=cells).local_blocks()
        dg = np.einsum("cii->ci", akk).reshape(-1)
        ref = precond.pjacobi_hl(k, dg, r_s, len(cells))
    else:
        hs = fdm.cell_lengths(mesh, cells)
        R = r_s.reshape(len(cells), n3)
        ref = np.concatenate([np.linalg.solve(fdm.block("hermite_like", k, cfg.eta, hs[i]), R[i])
                              for i in range(len(cells))])
    err = np.max(np.abs(z_s - ref)) / np.max(np.abs(ref))
    assert err <= 1e-12, err


def test_full_size_apply_pjacobi_on_sampled_cells():
    """The fused product and P^-1 (sipg_apply_pjacobi, the benchmark's step)
    on the headline mesh: y on sampled cells against the oracle's rows, and z
    on those cells against the oracle's P^-1 of the oracle's y (P^-1 acts
    cell by cell)."""
    torch, P = require_gpu()
    banner("full size apply_pjacobi")
    cfg = CONFIGS["scale_k4_64c_deformed"]
    mesh, k = cfg.mesh, cfg.degree
    n3 = (k + 1) ** 3
    op = P.Operator(mesh, k, cfg.eta)
    op.compute_gl_diagonal(return_diag=False)
    x = uniform_vector(op.ndofs, 0)
    xd = torch.from_numpy(x).cuda()
    y, z = op.apply_pjacobi(xd)
    torch.cuda.synchronize()
    cells = _sample_cells(mesh, 24, 5)
    y_s = _rows(y.cpu().numpy(), cells, n3)
    z_s = _rows(z.cpu().numpy(), cells, n3)
    del xd, y, z
    op.close()
    torch.cuda.empty_cache()
    ref_y = SIPG(mesh, k, cfg.eta, cells=cells).apply_naive(x)
    akk, _ = SIPG(mesh, k, cfg.eta, "nodal_gl", cells=cells).local_blocks()
    ref_z = precond.pjacobi_hl(k, np.einsum("cii->ci", akk).reshape(-1), ref_y, len(cells))
    err_y = np.max(np.abs(y_s - ref_y)) / np.max(np.abs(ref_y))
    err_z = np.max(np.abs(z_s - ref_z)) / np.max(np.abs(ref_z))
    assert err_y <= 1e-12 and err_z <= 1e-12, (err_y, err_z)


def test_largest_supported_size_on_sampled_cells():
    """2,097,152,000 unknowns (256^3 cells, k = 4, the paper's affine brick),
    just below the 2^31 limit of the in-kernel indices: the product on sampled
    cells (including the last ones) equals the oracle's rows."""
    torch, P = require_gpu()
    from workloads import paper_affine_brick
    banner("largest size 256^3 k=4 affine")
    mesh = paper_affine_brick(256)
    k = 4
    n3 = (k + 1) ** 3
    op = P.Operator(mesh, k, 2.0)
    assert op.ndofs == 256 ** 3 * n3 < 2 ** 31
    x = uniform_vector(op.ndofs, 0)
    xd = torch.from_numpy(x).cuda()
    y = op.apply(xd)
    torch.cuda.synchronize()
    cells = np.unique(np.concatenate([_sample_cells(mesh, 12, 4), [mesh.ncells - 2, mesh.ncells - 1]]))
    ys = y.view(-1, n3)[torch.from_numpy(cells).cuda()].cpu().numpy().reshape(-1)
    del xd, y
    op.close()
    torch.cuda.empty_cache()
    ref = SIPG(mesh, k, 2.0, cells=cells).apply_naive(x)
    err = np.max(np.abs(ys - ref)) / np.max(np.abs(ref))
    assert err <= 1e-12, err
