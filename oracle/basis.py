"""1D polynomial bases and Gauss quadrature on the reference interval (0, 1).

Test infrastructure (see oracle/__init__.py).  Every polynomial is kept in
product form  c * prod_l (xi - r_l)  and evaluated that way, never through
monomial coefficients (which lose accuracy quickly with the degree).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.special import roots_jacobi, eval_legendre


# --------------------------------------------------------------------------
# Product-form polynomials
# --------------------------------------------------------------------------
@dataclass
class ProductPoly:
    """p(xi) = c * prod(xi - roots); `reflect` evaluates p(1 - xi) instead."""

    c: float
    roots: np.ndarray
    reflect: bool = False

    def _raw(self, x):
        x = np.asarray(x, dtype=np.float64)
        out = np.full(x.shape, self.c, dtype=np.float64)
        for r in self.roots:
            out = out * (x - r)
        return out

    def _raw_deriv(self, x):
        # product rule: sum_k c prod_{l != k} (x - r_l)
        x = np.asarray(x, dtype=np.float64)
        out = np.zeros(x.shape, dtype=np.float64)
        for k in range(len(self.roots)):
            term = np.full(x.shape, self.c, dtype=np.float64)
            for l, r in enumerate(self.roots):
                if l != k:
                    term = term * (x - r)
            out = out + term
        return out

    def __call__(self, x):
        x = np.asarray(x, dtype=np.float64)
        return self._raw(1.0 - x) if self.reflect else self._raw(x)

    def deriv(self, x):
        x = np.asarray(x, dtype=np.float64)
        return -self._raw_deriv(1.0 - x) if self.reflect else self._raw_deriv(x)


class Basis1D:
    """A list of 1D polynomials phi_0..phi_p on (0, 1)."""

    def __init__(self, polys: List[ProductPoly], name: str):
        self.polys = polys
        self.name = name

    @property
    def degree(self) -> int:
        return len(self.polys) - 1

    def values(self, x) -> np.ndarray:
        """V[q, j] = phi_j(x_q)."""
        x = np.atleast_1d(np.asarray(x, dtype=np.float64))
        return np.stack([p(x) for p in self.polys], axis=1)

    def derivs(self, x) -> np.ndarray:
        """D[q, j] = phi_j'(x_q)."""
        x = np.atleast_1d(np.asarray(x, dtype=np.float64))
        return np.stack([p.deriv(x) for p in self.polys], axis=1)


# --------------------------------------------------------------------------
# Quadrature
# --------------------------------------------------------------------------
def gauss(nq: int):
    """Gauss-Legendre points and weights mapped from (-1, 1) to (0, 1)."""
    x, w = npleg.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


def jacobi_roots_01(m: int, a: float, b: float) -> np.ndarray:
    """Roots of the Jacobi polynomial P_m^{(a,b)}, mapped to (0, 1), ascending."""
    if m <= 0:
        return np.zeros(0)
    x, _ = roots_jacobi(m, a, b)
    return np.sort(0.5 * (x + 1.0))


def gauss_lobatto_points(n: int) -> np.ndarray:
    """The n Gauss-Lobatto points on [0, 1]: the end points and the roots of
    P'_{n-1}, which is proportional to the Jacobi polynomial P^{(1,1)}_{n-2}."""
    if n < 2:
        raise ValueError("Gauss-Lobatto needs n >= 2")
    return np.concatenate([[0.0], jacobi_roots_01(n - 2, 1.0, 1.0), [1.0]])


# --------------------------------------------------------------------------
# Hermite-like basis (Section 4.1, Appendix A)
# --------------------------------------------------------------------------
def hermite_like(p: int) -> Basis1D:
    """Hermite-like basis of degree p on (0, 1), Section 4.1.

    p = 1: the linear Lagrange pair {1 - xi, xi}.
    p = 2: {(1 - xi)^2, 2 xi (1 - xi), xi^2} (Appendix A).
    p >= 3: with r_l the p-3 roots of the Jacobi polynomial P^{4,4}_{p-3}
    mapped to (0, 1) and g(xi) = (xi - 1)^2 prod_l (xi - r_l),
        phi_0 = c0 (xi - xi1) g(xi),     phi_1 = c1 xi g(xi),
    where the free root xi1 makes phi_0 and phi_1 L2-orthogonal on (0, 1),
    c0 gives phi_0(0) = 1 and c1 gives phi_1'(0) = -phi_0'(0).  The bubbles
    phi_2..phi_{p-2} are xi^2 (xi - 1)^2 prod_{l != m} (xi - r_l), each scaled
    to one at its own node r_m (ordered by the node), and the last two
    functions mirror the first two: phi_{p-i}(xi) = phi_i(1 - xi).
    """
    if p < 1:
        raise ValueError("degree must be >= 1")
    if p == 1:
        return Basis1D([ProductPoly(-1.0, np.array([1.0])),
                        ProductPoly(1.0, np.array([0.0]))], "hermite_like")
    if p == 2:
        return Basis1D([ProductPoly(1.0, np.array([1.0, 1.0])),
                        ProductPoly(-2.0, np.array([0.0, 1.0])),
                        ProductPoly(1.0, np.array([0.0, 0.0]))], "hermite_like")
    r = jacobi_roots_01(p - 3, 4.0, 4.0)
    g_roots = np.concatenate([[1.0, 1.0], r])
    g = ProductPoly(1.0, g_roots)

    # Free root from  int_0^1 (xi - xi1) xi g(xi)^2 dxi = 0, a linear equation:
    # xi1 = int xi^2 g^2 / int xi g^2.  The integrands have degree <= 2p + 1,
    # so Gauss quadrature with p + 2 points is exact.
    xq, wq = gauss(p + 2)
    gq = g(xq)
    xi1 = np.sum(wq * xq * xq * gq * gq) / np.sum(wq * xq * gq * gq)

    g0 = g(np.array([0.0]))[0]
    dg0 = g.deriv(np.array([0.0]))[0]
    c0 = 1.0 / ((0.0 - xi1) * g0)                  # phi_0(0) = 1
    dphi0_0 = c0 * (g0 + (0.0 - xi1) * dg0)        # phi_0'(0)
    c1 = -dphi0_0 / g0                              # phi_1'(0) = c1 g(0) = -phi_0'(0)

    phi0 = ProductPoly(c0, np.concatenate([[xi1], g_roots]))
    phi1 = ProductPoly(c1, np.concatenate([[0.0], g_roots]))
    polys = [phi0, phi1]
    for m in range(p - 3):
        others = np.delete(r, m)
        roots = np.concatenate([[0.0, 0.0, 1.0, 1.0], others])
        val = ProductPoly(1.0, roots)(np.array([r[m]]))[0]
        polys.append(ProductPoly(1.0 / val, roots))
    polys.append(ProductPoly(c1, phi1.roots, reflect=True))
    polys.append(ProductPoly(c0, phi0.roots, reflect=True))
    return Basis1D(polys, "hermite_like")


def hermite_like_free_root(p: int) -> float:
    """The free root xi1 of phi_0 (p >= 3)."""
    return float(hermite_like(p).polys[0].roots[0])


# --------------------------------------------------------------------------
# Nodal Lagrange basis in the Gauss-Lobatto points (comparison basis)
# --------------------------------------------------------------------------
def lagrange(nodes: Sequence[float], name: str = "lagrange") -> Basis1D:
    nodes = np.asarray(nodes, dtype=np.float64)
    polys = []
    for j in range(len(nodes)):
        others = np.delete(nodes, j)
        c = 1.0 / np.prod(nodes[j] - others)
        polys.append(ProductPoly(c, others))
    return Basis1D(polys, name)


def nodal_gl(p: int) -> Basis1D:
    return lagrange(gauss_lobatto_points(p + 1), "nodal_gl")


def nodal_gauss(p: int) -> Basis1D:
    """Lagrange basis in the p+1 Gauss points: with the (p+1)-point Gauss rule
    the interpolation matrix S is the identity (collocation, Section 4.1)."""
    x, _ = gauss(p + 1)
    return lagrange(x, "nodal_gauss")


def make_basis(kind: str, p: int) -> Basis1D:
    if kind == "hermite_like":
        return hermite_like(p)
    if kind == "nodal_gl":
        return nodal_gl(p)
    if kind == "nodal_gauss":
        return nodal_gauss(p)
    raise ValueError(kind)


# --------------------------------------------------------------------------
# Rejected bases of Section 4.1 (only used as pins of Table 1)
# --------------------------------------------------------------------------
class _FuncBasis:
    def __init__(self, funcs):
        self.funcs = funcs

    def values(self, x):
        x = np.atleast_1d(np.asarray(x, dtype=np.float64))
        return np.stack([f(x) for f in self.funcs], axis=1)


def classical_hermite_cubic() -> _FuncBasis:
    """The four cubic Hermite polynomials of eq. (hermite_basic)."""
    return _FuncBasis([
        lambda x: 2 * x**3 - 3 * x**2 + 1,
        lambda x: x**3 - 2 * x**2 + x,
        lambda x: x**3 - x**2,
        lambda x: -2 * x**3 + 3 * x**2,
    ])


def hermite_legendre(p: int) -> _FuncBasis:
    """Cubic Hermite polynomials extended by the bubbles of eq.
    (hermite_legendre), 16 xi^2 (1 - xi)^2 sigma_m(xi), with sigma_m the
    orthonormal Legendre polynomial sqrt(2m+1) P_m(2 xi - 1), m = 0..p-4."""
    funcs = list(classical_hermite_cubic().funcs)
    for m in range(p - 3):
        funcs.append(lambda x, m=m: 16 * x**2 * (1 - x) ** 2
                     * np.sqrt(2 * m + 1) * eval_legendre(m, 2 * x - 1))
    return _FuncBasis(funcs)


# --------------------------------------------------------------------------
# 1D mass matrix and its condition number (Table 1)
# --------------------------------------------------------------------------
def mass_matrix(basis, p: int) -> np.ndarray:
    """M_ij = int_0^1 phi_i phi_j, exact with p + 2 Gauss points."""
    x, w = gauss(p + 2)
    V = basis.values(x)
    return V.T @ (w[:, None] * V)


def mass_condition_number(basis, p: int) -> float:
    """Spectral condition number lambda_max / lambda_min of the 1D mass matrix."""
    ev = np.linalg.eigvalsh(mass_matrix(basis, p))
    return float(ev[-1] / ev[0])


# --------------------------------------------------------------------------
# Reference-cell tables used by the matrix-free algorithm (Section 3)
# --------------------------------------------------------------------------
def face_rows(basis: Basis1D):
    """S_f and D_f at xi = 0 and xi = 1: values and first derivatives of all
    shape functions at the two end points."""
    e = np.array([0.0, 1.0])
    V = basis.values(e)
    D = basis.derivs(e)
    return V[0], D[0], V[1], D[1]
