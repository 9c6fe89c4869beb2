"""Reference-to-physical maps of the structured hexahedral meshes.

Test infrastructure (see oracle/__init__.py).  A mesh is described by a
`workloads.Mesh`; here the map F_K and its Jacobian are evaluated exactly
(analytically) at arbitrary reference points, in float64.

Cell K = (ix, iy, iz) has the lexicographic number ix + nx (iy + ny iz) and
    X = lo + ((ix, iy, iz) + xi) * h,   h = (hi - lo) / n
(on a graded brick, `mesh.width` = w: X_d = x_d(i_d) + xi_d (x_d(i_d + 1) - x_d(i_d))
with the cell boundaries x_d(i) = lo_d + i w_d for i < n_d and x_d(n_d) = hi_d)
    Y = L X
    F_K(xi) = Y + a s(Y) (1, 1, 1),      s(Y) = sin(pi Y1) sin(pi Y2) sin(pi Y3)
    J = dF_K/dxi = (I + a (1, 1, 1) grad s(Y)^T) L diag(h).
"""
from __future__ import annotations

import numpy as np


def _lin(mesh) -> np.ndarray:
    if mesh.lin is None:
        return np.eye(3)
    return np.asarray(mesh.lin, dtype=np.float64)


def cell_index(mesh, ix, iy, iz):
    nx, ny, _ = mesh.n
    return ix + nx * (iy + ny * iz)


def cell_coords(mesh, c):
    nx, ny, _ = mesh.n
    return c % nx, (c // nx) % ny, c // (nx * ny)


def cell_bounds(mesh, d: int) -> np.ndarray:
    """Cell boundaries x_d(0) < ... < x_d(n_d) of direction d of the brick."""
    n = int(mesh.n[d])
    lo, hi = float(mesh.lo[d]), float(mesh.hi[d])
    w = getattr(mesh, "width", None)
    if w is None:
        return lo + (hi - lo) * np.arange(n + 1) / n
    x = lo + float(w[d]) * np.arange(n + 1)
    x[n] = hi
    return x


def map_points(mesh, cells: np.ndarray, xi: np.ndarray):
    """Physical points and Jacobians.

    cells: int array [C]; xi: reference points [Q, 3].
    Returns x [C, Q, 3] and J [C, Q, 3, 3] with J[..., a, b] = dx_a / dxi_b.
    """
    cells = np.asarray(cells)
    idx = np.stack(cell_coords(mesh, cells), axis=-1)            # [C, 3]
    x0 = np.empty(idx.shape)
    h = np.empty(idx.shape)                                      # cell widths [C, 3]
    for d in range(3):
        b = cell_bounds(mesh, d)
        x0[:, d] = b[idx[:, d]]
        h[:, d] = b[idx[:, d] + 1] - b[idx[:, d]]
    X = x0[:, None, :] + xi[None, :, :] * h[:, None, :]          # [C, Q, 3]
    L = _lin(mesh)
    Y = X @ L.T                                                  # [C, Q, 3]
    LH = L[None, :, :] * h[:, None, :]                           # L diag(h) per cell [C, 3, 3]
    a = float(mesh.deform_amp)
    if a == 0.0:
        J = np.broadcast_to(LH[:, None], X.shape[:2] + (3, 3)).copy()
        return Y, J
    sn = np.sin(np.pi * Y)
    cs = np.cos(np.pi * Y)
    s = sn[..., 0] * sn[..., 1] * sn[..., 2]
    grad_s = np.pi * np.stack([cs[..., 0] * sn[..., 1] * sn[..., 2],
                               sn[..., 0] * cs[..., 1] * sn[..., 2],
                               sn[..., 0] * sn[..., 1] * cs[..., 2]], axis=-1)
    x = Y + a * s[..., None]
    dphi = np.eye(3) + a * np.ones(3)[:, None] * grad_s[..., None, :]  # [C,Q,3,3]
    J = dphi @ LH[:, None]
    return x, J
