"""Pins of the field-gather oracle: brute force, constants, exact reproduction of linear
fields, and the transpose relation with the deposition oracle."""
import numpy as np
import pytest

from oracle import deposit as od
from oracle.deposit import GUARD, PERIODIC, OracleGrid


def _parts(g, N, seed, margin=0.0):
    rng = np.random.default_rng(seed)
    pos = [rng.uniform(margin, g.n[d] - margin, N) for d in range(g.dim)]
    while len(pos) < 3:
        pos.append(np.zeros(N))
    return pos


def _fields(g, seed):
    rng = np.random.default_rng(seed)
    return ([rng.normal(size=g.shape) for _ in range(3)], [rng.normal(size=g.shape) for _ in range(3)])


@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("dim,bc,ng", [(3, PERIODIC, 0), (3, GUARD, 3), (2, PERIODIC, 0)])
def test_gather_matches_bruteforce(order, dim, bc, ng):
    g = OracleGrid(dim, (7, 6, 5)[:dim], order, bc=(bc,) * 3, ng=ng)
    pos = _parts(g, 30, seed=order + 10 * dim, margin=0.0 if bc == PERIODIC else 0.01)
    E, B = _fields(g, order)
    a = od.gather_fields(g, pos, E, B)
    b = od.gather_fields_bruteforce(g, pos, E, B)
    for c in range(3):
        np.testing.assert_allclose(a[0][c], b[0][c], rtol=0, atol=1e-12)
        np.testing.assert_allclose(a[1][c], b[1][c], rtol=0, atol=1e-12)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_gather_constant_fields(order):
    g = OracleGrid(3, (8, 7, 6), order)
    pos = _parts(g, 200, seed=order)
    E = [np.full(g.shape, v) for v in (1.5, -2.0, 0.25)]
    B = [np.full(g.shape, v) for v in (3.0, 0.5, -1.0)]
    Ep, Bp = od.gather_fields(g, pos, E, B)
    for c, v in enumerate((1.5, -2.0, 0.25)):
        np.testing.assert_allclose(Ep[c], v, rtol=1e-14)
    for c, v in enumerate((3.0, 0.5, -1.0)):
        np.testing.assert_allclose(Bp[c], v, rtol=1e-14)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_gather_reproduces_linear_fields(order):
    # B-splines reproduce linear functions: a field a + b x (x the node's own position,
    # with its half-cell shift) gathers to a + b x_p exactly, away from guard edges
    g = OracleGrid(3, (10, 9, 8), order, bc=(GUARD,) * 3, ng=3)
    pos = _parts(g, 100, seed=7 + order, margin=0.0)
    nodes = [np.arange(-3, g.n[d] + 3, dtype=np.float64) for d in range(3)]
    Z, Y, X = np.meshgrid(nodes[2], nodes[1], nodes[0], indexing="ij")
    E = [0.5 + 2.0 * (X + 0.5), -1.0 + 3.0 * (Y + 0.5), 0.25 - 1.5 * (Z + 0.5)]   # own-axis shift
    B = [0.5 + 2.0 * X, -1.0 + 3.0 * Y, 0.25 - 1.5 * Z]      # normal axis unshifted
    Ep, Bp = od.gather_fields(g, pos, E, B)
    np.testing.assert_allclose(Ep[0], 0.5 + 2.0 * pos[0], rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(Ep[1], -1.0 + 3.0 * pos[1], rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(Ep[2], 0.25 - 1.5 * pos[2], rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(Bp[0], 0.5 + 2.0 * pos[0], rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(Bp[1], -1.0 + 3.0 * pos[1], rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(Bp[2], 0.25 - 1.5 * pos[2], rtol=1e-13, atol=1e-12)


def test_gather_is_the_transpose_of_deposition():
    # <E_c, J_c(one particle)> = q w v_c E_c(x_p)
    g = OracleGrid(3, (9, 8, 7), 3, q=-1.0)
    pos = _parts(g, 1, seed=3)
    u = [np.array([0.3], np.float32), np.array([-0.2], np.float32), np.array([0.1], np.float32)]
    w = np.array([1.5], np.float32)
    E, B = _fields(g, 5)
    J = od.deposit(g, pos, u, w)
    Ep, _ = od.gather_fields(g, pos, E, B)
    _, v = od.velocity(u)
    for c in range(3):
        lhs = float((E[c] * J[c]).sum())
        rhs = float(g.q * np.float64(w[0]) * v[c][0] * Ep[c][0])
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(rhs))
