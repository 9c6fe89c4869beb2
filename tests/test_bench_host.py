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
