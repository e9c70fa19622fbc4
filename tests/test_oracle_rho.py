"""Pins of the charge-density oracle: brute force with the continuous B-spline kernels,
exact partition of unity, a closed form, and its tie to the 2D Jz (also nodal)."""
import numpy as np
import pytest

from oracle import deposit as od
from oracle.deposit import GUARD, PERIODIC, OracleGrid


def _parts(g, N, seed, margin=0.0):
    rng = np.random.default_rng(seed)
    pos = [rng.uniform(margin, g.n[d] - margin, N) for d in range(g.dim)]
    while len(pos) < 3:
        pos.append(np.zeros(N))
    w = rng.uniform(0.5, 2.0, N).astype(np.float32)
    return pos, w


@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("dim,bc,ng", [(3, PERIODIC, 0), (3, GUARD, 3), (2, PERIODIC, 0)])
def test_rho_matches_bruteforce(order, dim, bc, ng):
    n = (7, 6, 5)[:dim]
    g = OracleGrid(dim, n, order, q=-1.5, bc=(bc,) * 3, ng=ng)
    pos, w = _parts(g, 40, seed=order * 10 + dim, margin=0.0 if bc == PERIODIC else 0.01)
    a = od.deposit_rho(g, pos, w)
    b = od.deposit_rho_bruteforce(g, pos, w)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_rho_partition_of_unity(order):
    g = OracleGrid(3, (8, 7, 6), order, q=-1.0)
    pos, w = _parts(g, 500, seed=order)
    rho = od.deposit_rho(g, pos, w)
    assert abs(rho.sum() - g.q * w.astype(np.float64).sum()) <= 1e-10 * abs(w.sum())


def test_rho_closed_form_cubic_at_node():
    # order 3, particle exactly on node 3 of each axis: weights 1/6, 2/3, 1/6 per axis
    g = OracleGrid(3, (8, 8, 8), 3, q=2.0)
    pos = [np.array([3.0]), np.array([3.0]), np.array([3.0])]
    rho = od.deposit_rho(g, pos, np.array([1.0], np.float32))
    w1 = {2: 1 / 6, 3: 2 / 3, 4: 1 / 6}
    want = np.zeros(g.shape)
    for k, wz in w1.items():
        for j, wy in w1.items():
            for i, wx in w1.items():
                want[k, j, i] = 2.0 * wx * wy * wz
    np.testing.assert_allclose(rho, want, rtol=0, atol=1e-15)


def test_rho_is_2d_jz_over_vz():
    # in 2D, Jz is nodal in x and y, so with one common v_z it is v_z * rho
    g = OracleGrid(2, (9, 7), 3, q=-1.0)
    pos, w = _parts(g, 60, seed=5)
    N = len(w)
    uz = np.full(N, 0.4, np.float32)
    u = [np.zeros(N, np.float32), np.zeros(N, np.float32), uz]
    J = od.deposit(g, pos, u, w)
    vz = float(np.float64(uz[0]) / np.sqrt(1.0 + np.float64(uz[0]) ** 2))
    np.testing.assert_allclose(J[2], vz * od.deposit_rho(g, pos, w), rtol=1e-13, atol=1e-15)
