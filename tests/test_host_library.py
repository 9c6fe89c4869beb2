"""CPU-only checks of the HIP library's host side: it loads, exports every
symbol the header declares, its host-computed 1D tables match the oracle, the
launch shapes respect the gfx950 limits, and argument errors are reported
without touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import basis as b1d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
P = pytest.importorskip("paper_1907_08492_amd")


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sipg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sipg_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(P.lib, name), name
    assert set(P.EXPORTED) == set(names)


@pytest.mark.parametrize("basis", ["hermite_like", "nodal_gl", "nodal_gauss"])
@pytest.mark.parametrize("k", list(range(1, 9)))
def test_host_tables_match_oracle(basis, k):
    t = P.host_tables(k, basis)
    bas = b1d.make_basis(basis, k)
    x, w = b1d.gauss(k + 1)
    S, Sg = bas.values(x), bas.derivs(x)
    assert np.allclose(t["points"], x, atol=1e-15, rtol=0)
    assert np.allclose(t["weights"], w, atol=1e-15, rtol=0)
    assert np.max(np.abs(t["shape"] - S)) < 1e-14
    assert np.max(np.abs(t["shape_grad"] - Sg)) < 1e-14 * np.max(np.abs(Sg))
    # collocation derivative in the Gauss points reproduces S' = D S
    assert np.max(np.abs(t["colloc_grad"] @ S - Sg)) < 1e-13 * np.max(np.abs(Sg))
    s0, d0, s1, d1 = b1d.face_rows(bas)
    assert np.allclose(t["face_value0"], s0, atol=1e-14)
    assert np.allclose(t["face_value1"], s1, atol=1e-14)
    assert np.allclose(t["face_grad0"], d0, atol=1e-13 * np.max(np.abs(d0)))
    assert np.allclose(t["face_grad1"], d1, atol=1e-13 * np.max(np.abs(d1)))
    E = bas.values(b1d.gauss_lobatto_points(k + 1)).T
    assert np.allclose(t["to_gl"] @ E, np.eye(k + 1), atol=1e-12)


@pytest.mark.parametrize("k", list(range(1, 9)))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_launch_shape_limits(k, dtype):
    cpb, nt, lds = P.launch_shape(k, dtype)
    n = k + 1
    assert nt % 64 == 0 and nt <= 1024
    assert cpb * n * n <= nt          # one thread per pencil of every cell
    assert lds <= 160 * 1024          # LDS of one gfx950 compute unit
    assert cpb >= 1


def _xcd_remap(blk, nblk):
    """Model of the workgroup renumbering in the matrix-free kernel."""
    per = (nblk + 7) // 8
    xcd, slot = blk % 8, blk // 8
    full = 8 if nblk % 8 == 0 else nblk % 8
    start = xcd * per if xcd < full else full * per + (xcd - full) * (per - 1)
    return start + slot


@pytest.mark.parametrize("nblk", [1, 2, 7, 8, 9, 15, 16, 17, 63, 64, 65, 1000, 52429])
def test_xcd_remap_is_a_permutation(nblk):
    m = [_xcd_remap(b, nblk) for b in range(nblk)]
    assert sorted(m) == list(range(nblk))


@pytest.mark.parametrize("nblk,layer_blocks", [(1, 0), (9, 1), (100, 2), (100, 5), (128, 3), (1000, 7),
                                               (43691, 683), (7296, 96), (43691, 5000), (10923, 341),
                                               (22118, 461), (5, 1), (65, 3)])
def test_block_order_is_a_permutation(nblk, layer_blocks):
    """The kernel's own block order (sipg_host_block_order, the device
    function compiled for the host) visits every block exactly once."""
    m = P.host_block_order(nblk, layer_blocks)
    assert sorted(m.tolist()) == list(range(nblk))


def test_block_order_visits_z_neighbours_together():
    # 64^3 cells, 6 per block: each XCD's range holds 8 z-layers (P = 683
    # blocks each), visited column by column, so slots 8j .. 8j+7 of an XCD
    # are block j of 8 consecutive layers (the last column is one short), and
    # the blocks of one XCD form one contiguous range
    nblk, P_ = 43691, 683
    m = P.host_block_order(nblk, P_)
    for xcd in range(8):
        seq = m[xcd::8]
        assert seq.max() - seq.min() + 1 == len(seq)
        for j in range(0, 8 * 680, 8):
            assert all(seq[j + i + 1] - seq[j + i] == P_ for i in range(7))


def test_argument_errors_without_gpu():
    m = P.make_mesh(type("M", (), dict(n=(2, 2, 2), lo=(0, 0, 0), hi=(1, 1, 1)))())
    h = C.c_void_p()
    for deg, pen, basis, dt, geo in ((0, 1.0, 0, 0, 0), (9, 1.0, 0, 0, 0), (2, 0.0, 0, 0, 0),
                                     (2, 1.0, 5, 0, 0), (2, 1.0, 0, 7, 0), (2, 1.0, 0, 0, 9)):
        rc = P.lib.sipg_setup(C.byref(m), deg, pen, basis, dt, geo, None, None, C.byref(h))
        assert rc == -1, (deg, pen, basis, dt, geo)
        assert P.lib.sipg_last_error().decode()
    bad = P.make_mesh(type("M", (), dict(n=(2, 0, 2), lo=(0, 0, 0), hi=(1, 1, 1)))())
    assert P.lib.sipg_setup(C.byref(bad), 2, 1.0, 0, 0, 0, None, None, C.byref(h)) == -1
    deformed = P.make_mesh(type("M", (), dict(n=(2, 2, 2), lo=(0, 0, 0), hi=(1, 1, 1), deform_amp=0.1))())
    assert P.lib.sipg_setup(C.byref(deformed), 2, 1.0, 0, 0, 1, None, None, C.byref(h)) == -1
    assert P.lib.sipg_apply(None, None, None, None) == -1
    assert P.lib.sipg_basis_change(None, 0, None, None, None) == -1
    assert P.lib.sipg_ndofs(None) == -1
    assert P.lib.sipg_destroy(None) == 0
    assert P.lib.sipg_launch_shape(0, 0, None, None, None) == -1
    # more than 2^31 - 1 unknowns is rejected before any device work
    big = P.make_mesh(type("M", (), dict(n=(1300, 1300, 1300), lo=(0, 0, 0), hi=(1, 1, 1)))())
    assert P.lib.sipg_setup(C.byref(big), 1, 1.0, 0, 0, 0, None, None, C.byref(h)) == -1
    assert "too large" in P.lib.sipg_last_error().decode()
    assert P.lib.sipg_batch_create(0, None, None, None, C.byref(h)) == -1
    assert P.lib.sipg_batch_create(1, None, None, None, None) == -1
    null3 = (C.c_void_p * 1)(None)
    assert P.lib.sipg_batch_create(1, null3, null3, null3, C.byref(h)) == -1
    assert "entry 0" in P.lib.sipg_last_error().decode()
    assert P.lib.sipg_batch_apply(None, None) == -1
    assert P.lib.sipg_batch_get_info(None, None) == -1
    assert P.lib.sipg_batch_destroy(None) == 0


def test_single_hip_runtime_in_process():
    """The library binds to the HIP runtime PyTorch loaded (a second runtime in
    the same process does not see the device)."""
    maps = open("/proc/self/maps").read().splitlines()
    hip = {line.split()[-1] for line in maps if "libamdhip64" in line}
    assert len(hip) == 1, hip


@pytest.mark.parametrize("basis", ["hermite_like", "nodal_gl", "nodal_gauss"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 7, 8])
def test_host_fdm_tables_diagonalize_the_oracle_1d_matrices(basis, k):
    """The library's own 1D eigen-decomposition (Cholesky + Jacobi rotations)
    diagonalizes the oracle's interior-element SIPG and mass matrices:
    Z^T M Z = I, Z^T L Z = diag(lambda)."""
    from oracle import fdm
    for eta in (1.0, 2.0):
        zt, lam = P.host_fdm_tables(k, basis, eta)
        L, M = fdm.interior_1d(basis, k, 1.0, eta)
        Z = zt.T
        assert np.allclose(Z.T @ M @ Z, np.eye(k + 1), atol=1e-12)
        assert np.allclose(Z.T @ L @ Z, np.diag(lam), atol=1e-10 * np.max(np.abs(lam)))
        assert np.all(lam > 0)
        # reflection-even eigenvectors first, then the odd ones
        ne = k + 1 - (k + 1) // 2
        assert np.array_equal(zt[:ne], zt[:ne, ::-1])
        assert np.array_equal(zt[ne:], -zt[ne:, ::-1])


def test_graded_mesh_and_multigrid_option_errors_without_gpu():
    """Argument checks of the graded brick (sipg_mesh.width) and of the
    multigrid and server options are made before any device work."""
    from workloads import Mesh
    h = C.c_void_p()
    ok = P.make_mesh(Mesh(n=(3, 2, 2), width=(0.4, 0.6, 0.55)))
    for width in ((0.4, 0.6, 0.45),          # last cell of z wider than the others
                  (0.3, 0.6, 0.55),          # last cell of x wider (0.4 > 0.3)
                  (0.5, 0.6, 0.55),          # the first two x cells already reach hi
                  (-0.4, 0.6, 0.55)):
        bad = P.make_mesh(Mesh(n=(3, 2, 2), width=width))
        assert P.lib.sipg_setup(C.byref(bad), 2, 1.0, 0, 0, 0, None, None, C.byref(h)) == -1, width
        assert "graded brick" in P.lib.sipg_last_error().decode()
    B = P.binding
    o = B.SipgMgOpts()
    assert P.lib.sipg_mg_default_opts(C.byref(o)) == 0
    assert o.graded_coarsening == 0 and o.coarse_direct_max_dofs == 0
    for field, value in (("graded_coarsening", 2), ("coarse_direct_max_dofs", 5000), ("coarse_direct_max_dofs", -1)):
        o2 = B.SipgMgOpts()
        P.lib.sipg_mg_default_opts(C.byref(o2))
        setattr(o2, field, value)
        assert P.lib.sipg_mg_setup(C.byref(ok), 2, 2.0, 0, C.byref(o2), None, None, C.byref(h)) == -1, field
        assert "invalid options" in P.lib.sipg_last_error().decode()
    s = B.SipgServerOpts()
    assert P.lib.sipg_server_default_opts(C.byref(s)) == 0
    assert s.graded_coarsening == 0 and s.coarse_direct_max_dofs == 256
    s.coarse_direct_max_dofs = 5000
    assert P.lib.sipg_server_create(C.byref(s), None, C.byref(h)) == -1
    # grouping of same-problem requests into one multi-right-hand-side solve
    s = B.SipgServerOpts()
    P.lib.sipg_server_default_opts(C.byref(s))
    assert s.batch_max_rhs == 8 and s.batch_max_dofs == 1 << 20
    for field, value in (("batch_max_rhs", 0), ("batch_max_rhs", 17), ("batch_max_dofs", -1)):
        s2 = B.SipgServerOpts()
        P.lib.sipg_server_default_opts(C.byref(s2))
        setattr(s2, field, value)
        assert P.lib.sipg_server_create(C.byref(s2), None, C.byref(h)) == -1, field
        assert "batch_max_rhs" in P.lib.sipg_last_error().decode()


def test_solve_many_argument_errors_without_gpu():
    """sipg_mg_solve_many rejects null handles, bad right-hand-side counts and
    tolerances before any device work."""
    infos = (P.binding.SipgSolveInfo * 2)()
    assert P.lib.sipg_mg_solve_many(None, 2, None, None, 1e-8, 10, infos, None) == -1
    assert "null argument" in P.lib.sipg_last_error().decode()


def test_slab_argument_errors_without_gpu():
    from workloads import unit_cube
    h = C.c_void_p()
    m = P.make_mesh(unit_cube((2, 2, 4)))
    for z0, z1 in ((2, 2), (3, 1), (-1, 2), (0, 5)):
        assert P.lib.sipg_setup_slab(C.byref(m), z0, z1, 2, 2.0, 0, 0, 0, None, None, C.byref(h)) == -1, (z0, z1)
        assert "z0 < z1" in P.lib.sipg_last_error().decode()
    assert P.lib.sipg_apply_slab(None, None, None, None, None, None, None) == -1
    assert P.lib.sipg_pack_ghost(None, 0, None, None, None) == -1
    assert P.lib.sipg_ghost_size(None) == -1
