"""Pins of the charge-conserving (Esirkepov) oracle: the discrete continuity equation
against the nodal charge-density oracle, the total current of a uniform move, motion
along one axis, rest, and a hand-computed CIC case."""
import numpy as np
import pytest

from oracle import deposit as od
from oracle import esirkepov as oe
from oracle.deposit import GUARD, OracleGrid


def _move(g, seed, N=80, maxstep=0.9):
    rng = np.random.default_rng(seed)
    lo = [g.ng + 2.0 if g.bc[d] == GUARD else 0.0 for d in range(g.dim)]
    old = [rng.uniform(lo[d] + 1.0 if g.bc[d] == GUARD else 0.0,
                       g.n[d] - (1.0 if g.bc[d] == GUARD else 0.0), N) for d in range(g.dim)]
    step = [rng.uniform(-maxstep, maxstep, N) for _ in range(g.dim)]
    new = []
    for d in range(g.dim):
        x = old[d] + step[d]
        if g.bc[d] != GUARD:
            x = np.mod(x, g.n[d])
        new.append(x)
    u = [rng.normal(0, 0.4, N).astype(np.float32) for _ in range(3)]
    w = rng.uniform(0.5, 1.5, N)
    return old, new, step, u, w


def _div(g, J):
    div = np.zeros(g.shape)
    for d in range(g.dim):
        ax = g.dim - 1 - d                   # arrays are slowest-first
        div += (J[d] - np.roll(J[d], 1, axis=ax)) / g.dx[d]
    return div


@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("dim", [2, 3])
def test_continuity_equation(order, dim):
    n = (9, 8, 7)[:dim]
    g = OracleGrid(dim, n, order, dx=(1.0, 0.5, 2.0))
    old, new, _, u, w = _move(g, 100 * dim + order)
    # positions in physical units
    old = [old[d] * g.dx[d] for d in range(dim)]
    new = [new[d] * g.dx[d] for d in range(dim)]
    dt = 0.37
    J = oe.deposit_esirkepov(g, old, new, u, w, dt)
    r0 = od.deposit_rho(g, old, w)
    r1 = od.deposit_rho(g, new, w)
    resid = (r1 - r0) / dt + _div(g, J)
    assert np.max(np.abs(resid)) <= 1e-12 * np.max(np.abs(r1 - r0) / dt)


def test_continuity_with_guard_cells():
    g = OracleGrid(3, (10, 9, 8), 3, bc=(GUARD, GUARD, GUARD), ng=3)
    old, new, _, u, w = _move(g, 7)
    J = oe.deposit_esirkepov(g, old, new, u, w, 1.0)
    resid = (od.deposit_rho(g, new, w) - od.deposit_rho(g, old, w)) + _div(g, J)
    assert np.max(np.abs(resid)) <= 1e-12


@pytest.mark.parametrize("order", [1, 2, 3])
def test_total_current_is_charge_times_velocity(order):
    g = OracleGrid(3, (8, 8, 8), order, dx=(1.0, 1.5, 0.5))
    old, new, step, u, w = _move(g, 30 + order)
    old = [old[d] * g.dx[d] for d in range(3)]
    new = [new[d] * g.dx[d] for d in range(3)]
    dt = 0.8
    J = oe.deposit_esirkepov(g, old, new, u, w, dt)
    for d in range(3):
        want = g.q * np.sum(w * step[d] * g.dx[d]) / dt
        np.testing.assert_allclose(J[d].sum(), want, rtol=1e-12)


def test_2d_out_of_plane_current_total():
    g = OracleGrid(2, (12, 10), 2)
    old, new, _, u, w = _move(g, 5)
    J = oe.deposit_esirkepov(g, old, new, u, w, 0.5)
    _, v = od.velocity(u)
    np.testing.assert_allclose(J[2].sum(), g.q * np.sum(w * v[2]), rtol=1e-12)


def test_motion_along_x_gives_only_jx():
    g = OracleGrid(3, (8, 8, 8), 3)
    old, new, _, u, w = _move(g, 9)
    new = [new[0], old[1], old[2]]
    J = oe.deposit_esirkepov(g, old, new, u, w, 1.0)
    assert np.all(J[1] == 0) and np.all(J[2] == 0)
    assert np.abs(J[0]).max() > 0


def test_rest_gives_zero_current():
    g = OracleGrid(3, (6, 6, 6), 2)
    old, _, _, u, w = _move(g, 11)
    J = oe.deposit_esirkepov(g, old, old, u, w, 1.0)
    for c in range(3):
        assert np.all(J[c] == 0)


def test_cic_hand_computed():
    """Order 1, y and z on nodes, x from 2.25 to 2.75: half the charge moves from node 2
    to node 3, so the x face at 2.5 (storage index 2) carries q w (1/2) / dt."""
    g = OracleGrid(3, (6, 6, 6), 1)
    J = oe.deposit_esirkepov(g, [np.array([2.25]), np.array([3.0]), np.array([1.0])],
                             [np.array([2.75]), np.array([3.0]), np.array([1.0])],
                             [np.zeros(1, np.float32)] * 3, np.array([2.0]), 0.5)
    want = np.zeros(g.shape)
    want[1, 3, 2] = g.q * 2.0 * 0.5 / 0.5
    np.testing.assert_allclose(J[0], want, rtol=1e-14, atol=0)


def test_move_of_a_whole_cell_is_refused():
    g = OracleGrid(3, (6, 6, 6), 1)
    with pytest.raises(oe.MoveTooLarge):
        oe.deposit_esirkepov(g, [np.array([1.2])] * 3, [np.array([2.3]), np.array([1.2]),
                                                         np.array([1.2])],
                             [np.zeros(1, np.float32)] * 3, np.ones(1), 1.0)


def test_2d_out_of_plane_current_is_time_averaged_shape():
    """Order 1, moves inside one cell: the weights are linear in time along the path, and
    Jz must be q W v_z times the particle's shape averaged over the step (3-point
    Gauss-Legendre, exact for the quadratic product), computed from the charge-density
    oracle at intermediate positions."""
    g = OracleGrid(2, (10, 9), 1)
    rng = np.random.default_rng(44)
    N = 40
    cell = [rng.integers(0, g.n[d], N) for d in range(2)]
    a = [cell[d] + rng.uniform(0.05, 0.95, N) for d in range(2)]
    b = [np.clip(a[d] + rng.uniform(-0.3, 0.3, N), cell[d] + 0.01, cell[d] + 0.99)
         for d in range(2)]
    u = [rng.normal(0, 0.4, N).astype(np.float32) for _ in range(3)]
    w = rng.uniform(0.5, 1.5, N)
    J = oe.deposit_esirkepov(g, a, b, u, w, 0.6)
    _, v = od.velocity(u)
    t, wt = np.polynomial.legendre.leggauss(3)
    t, wt = 0.5 * (t + 1.0), 0.5 * wt
    want = sum(wk * od.deposit_rho(g, [a[d] + tk * (b[d] - a[d]) for d in range(2)], w * v[2])
               for tk, wk in zip(t, wt))
    np.testing.assert_allclose(J[2], want, rtol=0, atol=1e-13)
