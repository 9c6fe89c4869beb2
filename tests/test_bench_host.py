"""Host-side checks of the benchmark script (CPU): the algorithmic byte counts
it divides by, and its refusal of several GPUs."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from workloads import CONFIGS, unit_cube, paper_affine_brick  # noqa: E402


def _faces(n):
    nx, ny, nz = n
    return (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)


@pytest.mark.parametrize("cells,k,esz,per_point", [(64, 4, 8, True), (32, 7, 8, True), (48, 5, 4, True),
                                                   (64, 4, 8, False), (32, 7, 8, False)])
def test_algorithmic_bytes_per_unknown(cells, k, esz, per_point):
    # x read and y written once (2 values per unknown); 6 metric values per
    # cell quadrature point (or per cell) and 7 per face point (or per face)
    n = k + 1
    mesh = unit_cube(cells, 0.1) if per_point else paper_affine_brick(cells)
    ncells = cells ** 3
    ndofs = ncells * n ** 3
    metric = (6 * n ** 3 * ncells + 7 * n ** 2 * _faces(mesh.n)) if per_point else (6 * ncells + 7 * _faces(mesh.n))
    expected = esz * (2 + metric / ndofs)
    assert bench.alg_bytes_per_dof(mesh, k, esz, per_point) == pytest.approx(expected, rel=1e-14)


def test_headline_byte_count():
    # the headline workload: 64^3 deformed cells, k = 4, FP64
    cfg = CONFIGS["scale_k4_64c_deformed"]
    assert cfg.degree == 4 and tuple(cfg.mesh.n) == (64, 64, 64) and cfg.mesh.deformed
    b = bench.alg_bytes_per_dof(cfg.mesh, cfg.degree, 8, True)
    # 16 (x, y) + 48 (cell metric) + 8 * 7 * 25 * 798720 / 32768000 (face metric)
    assert b == pytest.approx(98.125, abs=1e-12)
    assert b * 32_768_000 == pytest.approx(3.2154e9, rel=1e-4)


def test_several_gpus_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


class _Counted:
    """A number that counts the floating-point operations applied to it (an
    FMA written as a * b + c counts 2, like the kernels' fused multiply-add)."""
    ops = 0

    def __init__(self, v):
        self.v = v

    def _op(self, o, f):
        _Counted.ops += 1
        return _Counted(f(self.v, o.v if isinstance(o, _Counted) else o))

    def __add__(self, o):
        return self._op(o, lambda a, b: a + b)

    __radd__ = __add__

    def __sub__(self, o):
        return self._op(o, lambda a, b: a - b)

    def __rsub__(self, o):
        return self._op(o, lambda a, b: b - a)

    def __mul__(self, o):
        return self._op(o, lambda a, b: a * b)

    __rmul__ = __mul__


def _even_odd_sweep(M, x, eps):
    """out = M x by the even-odd decomposition of a matrix with
    M[n-1-q][n-1-j] = eps M[q][j]: sums and differences of mirrored inputs,
    half-size products, and the outputs as their sum and difference."""
    n = len(x)
    h = n // 2
    e = [x[j] + x[n - 1 - j] for j in range(h)]
    o = [x[j] - x[n - 1 - j] for j in range(h)]
    out = [None] * n
    for q in range(h):
        ev = M[q][h] * x[h] if n % 2 else None
        od = None
        for j in range(h):
            a = (M[q][j] + M[q][n - 1 - j]) / 2
            b = (M[q][j] - M[q][n - 1 - j]) / 2
            ev = a * e[j] if ev is None else ev + a * e[j]
            od = b * o[j] if od is None else od + b * o[j]
        out[q] = ev + od
        out[n - 1 - q] = ev - od if eps > 0 else od - ev
    if n % 2:
        if eps > 0:
            m = M[h][h] * x[h]
            for j in range(h):
                m = m + (M[h][j] + M[h][n - 1 - j]) / 2 * e[j]
        else:
            m = None
            for j in range(h):
                t = (M[h][j] - M[h][n - 1 - j]) / 2 * o[j]
                m = t if m is None else m + t
        out[h] = m
    return out


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 8, 9])
@pytest.mark.parametrize("eps", [1, -1])
def test_even_odd_flop_count(n, eps):
    """The analytic FLOP count of one 1D sweep equals the operations of the
    even-odd algorithm counted one by one (a multiply followed by an add into
    an accumulator is the kernel's FMA: 2), and the sweep is correct."""
    import numpy as np
    rng = np.random.default_rng(n)
    A = rng.normal(size=(n, n))
    M = (A + eps * A[::-1, ::-1]) / 2          # M[n-1-q][n-1-j] = eps M[q][j]
    x = rng.normal(size=n)
    _Counted.ops = 0
    out = _even_odd_sweep(M.tolist(), [_Counted(v) for v in x], eps)
    assert np.allclose([o.v for o in out], M @ x)
    assert _Counted.ops == bench._eo_flops(n, eps)


def test_kernel_flop_counts_ordering():
    # per unknown: the per-point metric costs more than the per-cell one, the
    # diagonal-metric (reference-coordinate) cell term less, and the
    # Gauss-Lobatto basis (dense face rows) more than the Hermite-like one
    for k in (3, 4, 5, 7):
        q, c, d = (bench.kernel_flops_per_dof(k, "hermite_like", g) for g in ("qpoint", "cell", "diag"))
        assert d < c < q
        assert bench.kernel_flops_per_dof(k, "nodal_gl", "qpoint") > q
        assert bench.kernel_flops_per_dof(k, "hermite_like", "qpoint", "pjacobi") > q
