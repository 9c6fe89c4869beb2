"""Manufactured solutions, right-hand sides, interpolation and L2 errors.

Test infrastructure (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np

from . import basis as b1d
from .mesh import cell_bounds, cell_coords, map_points
from .sipg import tensor_eval


def sine(x):
    """u = sin(pi x) sin(pi y) sin(pi z); it vanishes on the unit cube's boundary."""
    return np.sin(np.pi * x[..., 0]) * np.sin(np.pi * x[..., 1]) * np.sin(np.pi * x[..., 2])


def sine_rhs(x):
    """f = -Laplace u = 3 pi^2 u for the sine solution."""
    return 3.0 * np.pi ** 2 * sine(x)


def quad_bubble(x):
    """u = x(1-x) y(1-y) z(1-z), a Q2 function vanishing on the unit cube's boundary."""
    q = x * (1.0 - x)
    return q[..., 0] * q[..., 1] * q[..., 2]


def quad_bubble_rhs(x):
    q = x * (1.0 - x)
    return 2.0 * (q[..., 1] * q[..., 2] + q[..., 0] * q[..., 2] + q[..., 0] * q[..., 1])


def modes_rhs(amps, waves):
    """f = sum_m a_m sin(p_m pi x) sin(q_m pi y) sin(r_m pi z) (a smooth RHS)."""
    amps = np.asarray(amps, dtype=np.float64)
    waves = np.asarray(waves, dtype=np.float64)

    def f(x):
        out = np.zeros(x.shape[:-1])
        for a, (p, q, r) in zip(amps, waves):
            out += a * (np.sin(p * np.pi * x[..., 0]) * np.sin(q * np.pi * x[..., 1])
                        * np.sin(r * np.pi * x[..., 2]))
        return out
    return f


def rhs(op, f, nq=None) -> np.ndarray:
    """b_i = sum_K sum_q f(F_K(xi_q)) phi_i(xi_q) det J w_q (cell-wise vector)."""
    nq = op.nq if nq is None else nq
    xq, wq = b1d.gauss(nq)
    g3, g2, g1 = np.meshgrid(xq, xq, xq, indexing="ij")
    pts = np.stack([g1.ravel(), g2.ravel(), g3.ravel()], axis=1)
    w3, w2, w1 = np.meshgrid(wq, wq, wq, indexing="ij")
    w = (w1 * w2 * w3).ravel()
    val, _ = tensor_eval(op.basis, pts)
    x, J = map_points(op.mesh, np.arange(op.ncells), pts)
    detJ = np.linalg.det(J)
    fx = f(x) * detJ * w                                     # [C, Q]
    return (fx @ val).reshape(-1)


def l2_error(op, uvec, u_exact, nq=None) -> float:
    """|| u_h - u ||_L2 with (k+3)^3 Gauss points per cell."""
    nq = op.k + 3 if nq is None else nq
    xq, wq = b1d.gauss(nq)
    g3, g2, g1 = np.meshgrid(xq, xq, xq, indexing="ij")
    pts = np.stack([g1.ravel(), g2.ravel(), g3.ravel()], axis=1)
    w3, w2, w1 = np.meshgrid(wq, wq, wq, indexing="ij")
    w = (w1 * w2 * w3).ravel()
    val, _ = tensor_eval(op.basis, pts)
    x, J = map_points(op.mesh, np.arange(op.ncells), pts)
    uh = np.asarray(uvec).reshape(op.ncells, -1) @ val.T
    err = (uh - u_exact(x)) ** 2 * np.linalg.det(J) * w
    return float(np.sqrt(err.sum()))


def interpolate_cartesian_product(op, funcs_1d) -> np.ndarray:
    """Coefficients of u(x) = prod_t g_t(x_t) on a Cartesian (unmapped) brick
    whose 1D factors g_t lie in P_k: on every cell each factor is matched at
    k+1 distinct points by solving the 1D collocation system of the basis."""
    mesh = op.mesh
    assert mesh.lin is None and mesh.deform_amp == 0.0
    n = op.n
    pts = b1d.gauss_lobatto_points(n)      # any n distinct points
    Vb = op.basis.values(pts)               # [n, n]
    bounds = [cell_bounds(mesh, t) for t in range(3)]
    out = np.zeros((op.ncells, n ** 3))
    ix, iy, iz = cell_coords(mesh, np.arange(op.ncells))
    idx = [ix, iy, iz]
    for c in range(op.ncells):
        coef = []
        for t in range(3):
            b = bounds[t]
            i = idx[t][c]
            xt = b[i] + pts * (b[i + 1] - b[i])
            coef.append(np.linalg.solve(Vb, funcs_1d[t](xt)))
        out[c] = np.einsum("a,b,c->cba", coef[0], coef[1], coef[2]).ravel()
    return out.reshape(-1)
