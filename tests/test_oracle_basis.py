"""Pins of the oracle's 1D bases and quadrature against what the paper prints
and what the mathematics fixes (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import basis as b1d

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _num(v, s=None):
    if isinstance(v, (int, float)):
        return float(v)
    expr = v.replace("s", repr(s)) if s is not None else v
    return float(eval(expr, {"sqrt": math.sqrt, "__builtins__": {}}))


def test_appendix_a_closed_forms():
    """Appendix A (p = 2..5) and Figure 1 (p = 3): the product-form basis equals
    the printed formulas at many points."""
    data = json.load(open(os.path.join(GOLDEN, "appendix_a_hermite_like.json")))
    x = np.linspace(0.0, 1.0, 101)
    s = math.sqrt(1.0 / 44.0)
    for p_str, funcs in data["bases"].items():
        p = int(p_str)
        V = b1d.hermite_like(p).values(x)
        for i, f in enumerate(funcs):
            ref = np.full_like(x, _num(f["scale"].replace("sqrt(44)", repr(math.sqrt(44)))
                                       if isinstance(f["scale"], str) else f["scale"]))
            for r in f["roots"]:
                ref = ref * (x - (_num(r.replace("s", repr(s))) if isinstance(r, str) else r))
            assert np.max(np.abs(V[:, i] - ref)) < 1e-13, (p, i)


def test_face_derivative_alpha_printed():
    data = json.load(open(os.path.join(GOLDEN, "appendix_a_hermite_like.json")))
    for p_str, alpha in data["face_derivative_alpha"].items():
        if p_str == "source":
            continue
        _, d0, _, _ = b1d.face_rows(b1d.hermite_like(int(p_str)))
        assert d0[0] == pytest.approx(-alpha, abs=1e-13)
        assert d0[1] == pytest.approx(alpha, abs=1e-13)


def test_figure2_p7_constants():
    """Figure 2: p = 7 nodes, free root and scale factors to three digits."""
    g = json.load(open(os.path.join(GOLDEN, "figure2_p7.json")))
    bas = b1d.hermite_like(7)
    xi1 = b1d.hermite_like_free_root(7)
    assert round(xi1, 4) == pytest.approx(g["free_root"], abs=6e-5)
    assert round(1.0 - xi1, 3) == pytest.approx(g["mirrored_free_root"], abs=6e-4)
    nodes = b1d.jacobi_roots_01(4, 4.0, 4.0)
    assert np.allclose(np.round(nodes, 3), g["interior_nodes"], atol=1e-12)
    # scale factors: leading coefficient of each product-form polynomial
    # (the mirrored ones carry a sign (-1)^degree from xi -> 1 - xi)
    for i in range(8):
        poly = bas.polys[i]
        lead = poly.c * ((-1.0) ** len(poly.roots) if poly.reflect else 1.0)
        ref = g["scales"][f"phi{i}"]
        assert abs(lead - ref) <= 0.5 * 10 ** (math.floor(math.log10(abs(ref))) - 2) + 1e-9, (i, lead)


def test_table1_condition_numbers():
    """Table 1: mass-matrix condition numbers, all three columns, p = 3..30."""
    t = json.load(open(os.path.join(GOLDEN, "table1_condition_numbers.json")))
    for p_str, (hleg, hl, gl) in t["rows"].items():
        p = int(p_str)
        got = [b1d.mass_condition_number(b1d.hermite_legendre(p), p),
               b1d.mass_condition_number(b1d.hermite_like(p), p),
               b1d.mass_condition_number(b1d.nodal_gl(p), p)]
        for g_, r in zip(got, (hleg, hl, gl)):
            # three printed digits: within one unit of the last printed digit
            # (covers rounding and truncation of the printed value)
            unit = 10.0 ** (math.floor(math.log10(r)) - 2)
            assert abs(g_ - r) <= unit, (p, g_, r)


@pytest.mark.parametrize("p", list(range(1, 13)))
def test_face_property(p):
    """S_f = [1, 0, ...], D_f = [-alpha, alpha, 0, ...] at xi = 0, mirrored at 1
    (eq. hermite_relaxed and Section 4.1, item 3)."""
    s0, d0, s1, d1 = b1d.face_rows(b1d.hermite_like(p))
    e0 = np.zeros(p + 1)
    e0[0] = 1.0
    assert np.allclose(s0, e0, atol=1e-13)
    assert np.allclose(s1, e0[::-1], atol=1e-13)
    alpha = d0[1]
    assert alpha > 0
    ref = np.zeros(p + 1)
    ref[0], ref[1] = -alpha, alpha
    assert np.allclose(d0, ref, atol=1e-11 * alpha)
    assert np.allclose(d1, -ref[::-1], atol=1e-11 * alpha)


@pytest.mark.parametrize("p", list(range(1, 13)))
def test_partition_of_unity_and_symmetry(p):
    """u = [1, ..., 1] represents u_h = 1; phi_i(xi) = phi_{p-i}(1 - xi)."""
    bas = b1d.hermite_like(p)
    x = np.linspace(0, 1, 57)
    V = bas.values(x)
    assert np.max(np.abs(V.sum(axis=1) - 1.0)) < 1e-13
    assert np.max(np.abs(bas.derivs(x).sum(axis=1))) < 1e-11
    assert np.max(np.abs(V - bas.values(1.0 - x)[:, ::-1])) < 1e-13


@pytest.mark.parametrize("p", [3, 4, 5, 7, 10, 15])
def test_orthogonality_rules(p):
    """int phi_0 phi_1 = 0 (the rule fixing the free root) and the bubbles are
    mutually L2-orthogonal (nodes are roots of P^{4,4}_{p-3})."""
    M = b1d.mass_matrix(b1d.hermite_like(p), p)
    scale = np.max(np.abs(M))
    assert abs(M[0, 1]) < 1e-14 * scale * 10
    for i in range(2, p - 1):
        for j in range(2, p - 1):
            if i != j:
                assert abs(M[i, j]) < 1e-13 * scale, (i, j)


def test_gauss_quadrature_exactness():
    for nq in range(1, 10):
        x, w = b1d.gauss(nq)
        for m in range(2 * nq):
            assert abs(np.sum(w * x ** m) - 1.0 / (m + 1)) < 1e-14
        # the first non-integrable monomial is not exact
        assert abs(np.sum(w * x ** (2 * nq)) - 1.0 / (2 * nq + 1)) > 1e-12


def test_gauss_lobatto_points_and_lagrange():
    for n in range(2, 10):
        x = b1d.gauss_lobatto_points(n)
        assert x[0] == 0.0 and x[-1] == 1.0
        assert np.allclose(x, 1.0 - x[::-1], atol=1e-14)
        V = b1d.nodal_gl(n - 1).values(x)
        assert np.allclose(V, np.eye(n), atol=1e-13)
    # n = 3: the mid point; n = 4: (1 +- 1/sqrt5)/2 (roots of P'_3)
    assert np.allclose(b1d.gauss_lobatto_points(3), [0, 0.5, 1])
    assert np.allclose(b1d.gauss_lobatto_points(4)[1:3],
                       [(1 - 1 / math.sqrt(5)) / 2, (1 + 1 / math.sqrt(5)) / 2])


def test_classical_hermite_condition_p3():
    """Table 1 first entry also equals the classical cubic Hermite basis."""
    c = b1d.mass_condition_number(b1d.classical_hermite_cubic(), 3)
    assert abs(c - 1.06e3) <= 10.0


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8])
def test_nodal_gauss_collocation_and_diagonal_mass(p):
    """Section 4.1: with nodes at the p+1 Gauss points, S = I and (Gauss being
    exact to degree 2p+1) the exact mass matrix is diag(weights); the face rows
    S_f are dense."""
    bas = b1d.make_basis("nodal_gauss", p)
    x, w = b1d.gauss(p + 1)
    assert np.allclose(bas.values(x), np.eye(p + 1), atol=1e-13)
    xe, we = b1d.gauss(p + 3)
    V = bas.values(xe)
    M = V.T @ (we[:, None] * V)
    assert np.allclose(M, np.diag(w), atol=1e-14)
    v0 = bas.values([0.0])[0]
    assert np.all(np.abs(v0) > 1e-3) and abs(v0.sum() - 1.0) < 1e-13
