"""Reference-to-physical maps of the structured hexahedral meshes.

Test infrastructure (see oracle/__init__.py).  A mesh is described by a
`workloads.Mesh`; here the map F_K and its Jacobian are evaluated exactly
(analytically) at arbitrary reference points, in float64.

Cell K = (ix, iy, iz) has the lexicographic number ix + nx (iy + ny iz) and
    X = lo + ((ix, iy, iz) + xi) * h,   h = (hi - lo) / n
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


def map_points(mesh, cells: np.ndarray, xi: np.ndarray):
    """Physical points and Jacobians.

    cells: int array [C]; xi: reference points [Q, 3].
    Returns x [C, Q, 3] and J [C, Q, 3, 3] with J[..., a, b] = dx_a / dxi_b.
    """
    cells = np.asarray(cells)
    lo = np.asarray(mesh.lo, dtype=np.float64)
    hi = np.asarray(mesh.hi, dtype=np.float64)
    n = np.asarray(mesh.n, dtype=np.float64)
    h = (hi - lo) / n
    ix, iy, iz = cell_coords(mesh, cells)
    idx = np.stack([ix, iy, iz], axis=-1).astype(np.float64)     # [C, 3]
    X = lo + (idx[:, None, :] + xi[None, :, :]) * h              # [C, Q, 3]
    L = _lin(mesh)
    Y = X @ L.T                                                  # [C, Q, 3]
    LH = L * h[None, :]                                          # L diag(h)
    a = float(mesh.deform_amp)
    if a == 0.0:
        J = np.broadcast_to(LH, X.shape[:2] + (3, 3)).copy()
        return Y, J
    sn = np.sin(np.pi * Y)
    cs = np.cos(np.pi * Y)
    s = sn[..., 0] * sn[..., 1] * sn[..., 2]
    grad_s = np.pi * np.stack([cs[..., 0] * sn[..., 1] * sn[..., 2],
                               sn[..., 0] * cs[..., 1] * sn[..., 2],
                               sn[..., 0] * sn[..., 1] * cs[..., 2]], axis=-1)
    x = Y + a * s[..., None]
    dphi = np.eye(3) + a * np.ones(3)[:, None] * grad_s[..., None, :]  # [C,Q,3,3]
    J = dphi @ LH
    return x, J
