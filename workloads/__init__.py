"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module holds only *input definitions*: mesh descriptions (brick bounds,
cell counts, an optional linear map, a deformation amplitude), degrees,
penalty factors and seeded random vectors.  It contains none of the
method's arithmetic (no basis functions, no geometry evaluation, no
integrals); the oracle and the GPU library each implement those on their own.

Every workload follows the setups of the paper:
  * the affine benchmark brick (-0.95,0.95)x(-0.9,0.89)x(-0.85,0.83) mapped by
    the constant Jacobian of Section 5;
  * the unit cube with the sine deformation x += a*sin(pi x)sin(pi y)sin(pi z)
    applied to every coordinate (the deformed-mesh case of the data-access
    model of Section 4.2, here with stored per-quadrature-point metric terms);
  * the unit cube without deformation (Cartesian), used for the manufactured
    solution u = sin(pi x) sin(pi y) sin(pi z) (Section 6.2 uses a sine too).
"""
from __future__ import annotations

from dataclasses import dataclass, field, asdict
from typing import Optional, Sequence, Tuple

import numpy as np

# Constant Jacobian of the affine benchmark geometry (Section 5).
PAPER_LINEAR_MAP = (
    (1.12, 0.24, 0.36),
    (0.24, 1.36, 0.48),
    (0.36, 0.48, 1.60),
)
PAPER_BRICK_LO = (-0.95, -0.9, -0.85)
PAPER_BRICK_HI = (0.95, 0.89, 0.83)


@dataclass(frozen=True)
class Mesh:
    """A structured brick of n[0] x n[1] x n[2] hexahedra.

    The reference-to-physical map of cell (ix, iy, iz) is
        X(xi) = lo + ((ix, iy, iz) + xi) * (hi - lo) / n     (brick point)
        Y     = L X                                        (linear map, L = I if None)
        Z     = Y + deform_amp * sin(pi Y1) sin(pi Y2) sin(pi Y3) * (1, 1, 1)
    With `width` = (w1, w2, w3) the brick is graded instead: in direction d the
    cells 0 .. n_d - 2 have width w_d and the last one ends at hi_d (its width
    hi_d - lo_d - (n_d - 1) w_d lies in (0, w_d]).
    """

    n: Tuple[int, int, int]
    lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    hi: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    lin: Optional[Tuple[Tuple[float, float, float], ...]] = None
    deform_amp: float = 0.0
    width: Optional[Tuple[float, float, float]] = None

    @property
    def ncells(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def deformed(self) -> bool:
        return self.deform_amp != 0.0

    def asdict(self) -> dict:
        return asdict(self)


def unit_cube(n: int | Sequence[int], deform_amp: float = 0.0) -> Mesh:
    if isinstance(n, int):
        n = (n, n, n)
    return Mesh(n=tuple(int(v) for v in n), deform_amp=float(deform_amp))


def paper_affine_brick(n: int | Sequence[int]) -> Mesh:
    if isinstance(n, int):
        n = (n, n, n)
    return Mesh(n=tuple(int(v) for v in n), lo=PAPER_BRICK_LO, hi=PAPER_BRICK_HI,
                lin=PAPER_LINEAR_MAP)


@dataclass(frozen=True)
class Operator:
    """An SIPG operator configuration: mesh, degree k, penalty factor eta, basis."""

    mesh: Mesh
    degree: int
    eta: float = 2.0
    basis: str = "hermite_like"  # or "nodal_gl"

    @property
    def ndofs(self) -> int:
        return self.mesh.ncells * (self.degree + 1) ** 3


def uniform_vector(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """x ~ U[-1, 1], numpy default_rng(seed), drawn in float64 and then cast."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=int(n)).astype(dtype)


# Named workloads.  "small" is the correctness case (8^3 Cartesian unit cube,
# k=3, eta=2); the "scale_*" cases are the large matvec measurements.
CONFIGS = {
    "small_k3_8c": Operator(unit_cube(8), 3, 2.0),
    "scale_k4_64c_affine": Operator(paper_affine_brick(64), 4, 2.0),
    "scale_k4_64c_deformed": Operator(unit_cube(64, 0.1), 4, 2.0),
    "scale_k7_32c_affine": Operator(paper_affine_brick(32), 7, 2.0),
    "scale_k7_32c_deformed": Operator(unit_cube(32, 0.1), 7, 2.0),
    "mixed_k5_48c_deformed": Operator(unit_cube(48, 0.1), 5, 2.0),
}


def with_basis(op: Operator, basis: str) -> Operator:
    return Operator(op.mesh, op.degree, op.eta, basis)


def batch_operators(count: int = 256, seed: int = 0):
    """Independent operators applied together: cube of n^3 cells with
    n ~ U{4..24} and degree k ~ U{2..7} (numpy default_rng(seed)); the first
    half on the affine benchmark brick, the second half on the sine-deformed
    unit cube (amplitude 0.1).  Operator i takes x = uniform_vector(., i)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(4, 25, size=count)
    ks = rng.integers(2, 8, size=count)
    out = []
    for i in range(count):
        n, k = int(ns[i]), int(ks[i])
        mesh = paper_affine_brick(n) if i < count // 2 else unit_cube(n, 0.1)
        out.append(Operator(mesh, k, 2.0))
    return out


def serving_requests(rate_per_s: float = 200.0, seconds: float = 60.0, seed: int = 0):
    """Poisson arrivals of Poisson solves: unit cube with n^3 cells,
    n = round(exp(U[ln 8, ln 48])), degree k ~ U{3, 4, 5}, source
    f = sum_{m<8} a_m sin(p_m pi x) sin(q_m pi y) sin(r_m pi z) with
    a_m ~ N(0, 1) and (p, q, r)_m ~ U{1..4}^3.  Returns a list of
    (arrival_time_s, n, k, amps[8], waves[8][3])."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= seconds:
            break
        n = int(round(np.exp(rng.uniform(np.log(8.0), np.log(48.0)))))
        k = int(rng.integers(3, 6))
        amps = rng.normal(size=8)
        waves = rng.integers(1, 5, size=(8, 3))
        out.append((t, n, k, amps, waves))
    return out
