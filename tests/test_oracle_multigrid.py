"""Pin of the oracle's nested-mesh embedding: the fine representation of a
coarse function takes the same values at every point (CPU only)."""
import numpy as np
import pytest

from oracle import multigrid as omg
from oracle.sipg import tensor_eval
from oracle import basis as b1d
from oracle.mesh import cell_bounds
from workloads import Mesh, unit_cube


@pytest.mark.parametrize("kind", ["hermite_like", "nodal_gl"])
@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_embedding_reproduces_coarse_function(kind, k):
    n = k + 1
    rng = np.random.default_rng(k)
    coarse = rng.uniform(-1, 1, n ** 3)                 # one coarse cell
    fine = omg.prolongate(coarse, (2, 2, 2), kind, k).reshape(8, n ** 3)
    bas = b1d.make_basis(kind, k)
    pts = rng.uniform(0, 1, (50, 3))                    # child reference points
    vf, _ = tensor_eval(bas, pts)
    for child in range(8):
        s = np.array([child % 2, (child // 2) % 2, child // 4])
        vc, _ = tensor_eval(bas, 0.5 * (s + pts))       # same points in the coarse cell
        assert np.max(np.abs(vf @ fine[child] - vc @ coarse)) < 1e-12


def test_restriction_is_transpose():
    k, nc = 2, (4, 2, 2)
    n3 = (k + 1) ** 3
    rng = np.random.default_rng(0)
    c = rng.uniform(-1, 1, (nc[0] // 2) * (nc[1] // 2) * (nc[2] // 2) * n3)
    f = rng.uniform(-1, 1, nc[0] * nc[1] * nc[2] * n3)
    lhs = omg.prolongate(c, nc, "hermite_like", k) @ f
    rhs = c @ omg.restrict(f, nc, "hermite_like", k)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("kind", ["hermite_like", "nodal_gl", "nodal_gauss"])
@pytest.mark.parametrize("kf,kc", [(2, 1), (3, 1), (4, 2), (5, 2), (7, 3), (8, 4), (5, 4)])
def test_degree_embedding_reproduces_coarse_function(kind, kf, kc):
    """The degree-kf coefficients from p_prolongate define the same function as
    the degree-kc ones at random points; restriction is the transpose."""
    rng = np.random.default_rng(kf * 10 + kc)
    c = rng.uniform(-1, 1, 2 * (kc + 1) ** 3)
    f = omg.p_prolongate(c, 2, kind, kf, kc).reshape(2, (kf + 1) ** 3)
    pts = rng.uniform(0, 1, (40, 3))
    vf, _ = tensor_eval(b1d.make_basis(kind, kf), pts)
    vc, _ = tensor_eval(b1d.make_basis(kind, kc), pts)
    for cell in range(2):
        ref = vc @ c.reshape(2, -1)[cell]
        assert np.max(np.abs(vf @ f[cell] - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))
    g = rng.uniform(-1, 1, 2 * (kf + 1) ** 3)
    lhs = omg.p_prolongate(c, 2, kind, kf, kc) @ g
    rhs = c @ omg.p_restrict(g, 2, kind, kf, kc)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


# graded coarsening of a 5 x 4 x 3 unit cube: fine cells paired from 0 on, the
# last one alone for odd counts (twice the regular width)
GRADED_CHAIN = [unit_cube((5, 4, 3)),
                Mesh(n=(3, 2, 2), width=(0.4, 0.5, 2 / 3)),
                Mesh(n=(2, 1, 1), width=(0.8, 1.0, 4 / 3))]


def _eval_on_brick(mesh, kind, k, coef, pts):
    """Values of the function with coefficients coef at physical points of a
    Cartesian brick (cell found from the cell bounds)."""
    bas = b1d.make_basis(kind, k)
    n3 = (k + 1) ** 3
    out = np.empty(len(pts))
    for p_i, x in enumerate(pts):
        idx, xi = [], []
        for d in range(3):
            b = cell_bounds(mesh, d)
            i = min(int(np.searchsorted(b, x[d])) - 1, len(b) - 2)
            i = max(i, 0)
            idx.append(i)
            xi.append((x[d] - b[i]) / (b[i + 1] - b[i]))
        c = idx[0] + mesh.n[0] * (idx[1] + mesh.n[1] * idx[2])
        v, _ = tensor_eval(bas, np.array([xi]))
        out[p_i] = v[0] @ coef[c * n3:(c + 1) * n3]
    return out


@pytest.mark.parametrize("kind", ["hermite_like", "nodal_gl"])
@pytest.mark.parametrize("k", [1, 2, 4])
@pytest.mark.parametrize("level", [0, 1])
def test_nested_embedding_reproduces_coarse_function(kind, k, level):
    """On the graded chain (odd counts: one child; unequal pairs on the
    second step) the fine coefficients of a coarse function take its values
    at random points, and the restriction is the transpose."""
    fine, coarse = GRADED_CHAIN[level], GRADED_CHAIN[level + 1]
    n3 = (k + 1) ** 3
    rng = np.random.default_rng(10 * k + level)
    c = rng.uniform(-1, 1, coarse.ncells * n3)
    f = omg.prolongate_nested(c, fine, coarse, kind, k)
    pts = rng.uniform(0, 1, (60, 3))
    ref = _eval_on_brick(coarse, kind, k, c, pts)
    assert np.max(np.abs(_eval_on_brick(fine, kind, k, f, pts) - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))
    g = rng.uniform(-1, 1, fine.ncells * n3)
    lhs = f @ g
    rhs = c @ omg.restrict_nested(g, fine, coarse, kind, k)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("k", [1, 3])
def test_nested_embedding_equals_halving_on_even_bricks(k):
    rng = np.random.default_rng(k)
    c = rng.uniform(-1, 1, 2 * 1 * 3 * (k + 1) ** 3)
    a = omg.prolongate_nested(c, unit_cube((4, 2, 6)), unit_cube((2, 1, 3)), "hermite_like", k)
    assert np.max(np.abs(a - omg.prolongate(c, (4, 2, 6), "hermite_like", k))) < 1e-13
