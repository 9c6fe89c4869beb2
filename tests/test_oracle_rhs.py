"""Pins of the oracle's right-hand side for a sum of sine modes (CPU).

On a Cartesian brick the map is x_t = lo_t + (i_t + xi_t) h_t per axis, so for
one mode a sin(p pi x) sin(q pi y) sin(r pi z) the load vector
b_i = int f phi_i factorises into 1D load vectors, one per axis, combined as
a Kronecker product in the cell-wise layout (cell = ix + nx (iy + ny iz),
local index i1 + n (i2 + n i3)).  The 1D integrals are computed here with a
40-point Gauss rule of numpy (exact to rounding for these smooth
integrands), independently of the oracle's 3D quadrature loop.  Distinct wave
numbers per axis catch a transposed axis; several modes catch a wrong
amplitude or summation.
"""
import numpy as np
import pytest

from oracle import basis as b1d
from oracle import mms
from oracle.sipg import SIPG
from workloads import Mesh, unit_cube


def _load_1d(basis, k, ncell, lo, h, w):
    """[ncell, k+1] integrals of sin(w pi x) phi_i((x - lo)/h - cell) over each cell."""
    xg, wg = np.polynomial.legendre.leggauss(40)
    xi = 0.5 * (xg + 1.0)
    wt = 0.5 * wg
    phi = basis.values(xi)              # [q, i]
    out = np.zeros((ncell, k + 1))
    for c in range(ncell):
        x = lo + (c + xi) * h
        out[c] = (np.sin(w * np.pi * x) * wt * h) @ phi
    return out


def _kron_rhs(mesh, k, kind, amps, waves):
    basis = b1d.make_basis(kind, k)
    nx, ny, nz = mesh.n
    lo = np.asarray(mesh.lo, float)
    h = (np.asarray(mesh.hi, float) - lo) / np.asarray(mesh.n, float)
    n = k + 1
    b = np.zeros((nz, ny, nx, n, n, n))      # [iz, iy, ix, i3, i2, i1]
    for a, (p, q, r) in zip(amps, waves):
        bx = _load_1d(basis, k, nx, lo[0], h[0], p)
        by = _load_1d(basis, k, ny, lo[1], h[1], q)
        bz = _load_1d(basis, k, nz, lo[2], h[2], r)
        b += a * np.einsum("zc,yb,xa->zyxcba", bz, by, bx)
    return b.reshape(-1)


@pytest.mark.parametrize("kind", ["hermite_like", "nodal_gl"])
@pytest.mark.parametrize("k", [2, 3, 4])
def test_modes_rhs_factorises_cartesian(kind, k):
    mesh = Mesh(n=(3, 2, 4), lo=(0.0, 0.0, 0.0), hi=(1.0, 0.5, 2.0))
    amps = [0.7, -1.3, 2.1]
    waves = [(1, 2, 3), (3, 1, 2), (2, 4, 1)]
    op = SIPG(mesh, k, 2.0, kind)
    # a Gauss rule with k+8 points per direction integrates the product of the
    # basis (degree k) and the sines (|w| <= 4 over cells of size <= 1/2)
    # to near rounding
    b = mms.rhs(op, mms.modes_rhs(amps, waves), nq=k + 8)
    ref = _kron_rhs(mesh, k, kind, amps, waves)
    assert np.max(np.abs(b - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_modes_rhs_single_mode_is_sine_rhs():
    """The mode (1,1,1) with amplitude 3 pi^2 is the manufactured source
    f = -Laplace(sin sin sin), pinned by the convergence tests."""
    x = np.random.default_rng(0).uniform(0.0, 1.0, (50, 3))
    f = mms.modes_rhs([3 * np.pi ** 2], [(1, 1, 1)])
    assert np.allclose(f(x), mms.sine_rhs(x), rtol=0, atol=1e-13)


def test_modes_rhs_default_rule_close_to_exact():
    """With the operator's own k+1 point rule the load vector differs from the
    exact integrals only by the quadrature error, which falls with h."""
    amps, waves = [1.0, -0.5], [(1, 2, 1), (2, 1, 3)]
    errs = []
    for m in (4, 8):
        mesh = unit_cube(m)
        op = SIPG(mesh, 3, 2.0)
        b = mms.rhs(op, mms.modes_rhs(amps, waves))
        ref = _kron_rhs(mesh, 3, "hermite_like", amps, waves)
        errs.append(np.max(np.abs(b - ref)) / np.max(np.abs(ref)))
    assert errs[1] < errs[0] / 8
