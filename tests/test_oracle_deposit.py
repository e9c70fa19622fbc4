"""Pins of the deposition oracle (Eq. 1) against closed forms, invariants and brute force."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import deposit as od
from oracle.deposit import GUARD, PERIODIC, OracleGrid
from paper_2601_08277_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand_particles(g, N, seed, u_sigma=0.3, margin=0.0):
    rng = np.random.default_rng(seed)
    pos = [rng.uniform(margin, g.n[d] - margin, N) for d in range(g.dim)]
    while len(pos) < 3:
        pos.append(np.zeros(N))
    u = [rng.normal(0, u_sigma, N).astype(np.float32) for _ in range(3)]
    w = rng.uniform(0.5, 2.0, N).astype(np.float32)
    return pos, u, w


def test_golden_single_particle_cic():
    g = OracleGrid(3, (5, 6, 4), order=1, q=-1.0)
    pos = [np.array([2.25]), np.array([3.5]), np.array([1.75])]
    u = [np.array([0.75], np.float32), np.zeros(1, np.float32), np.zeros(1, np.float32)]
    w = np.array([2.0], np.float32)
    J = od.deposit(g, pos, u, w)
    want = np.zeros((3,) + g.shape)
    with open(os.path.join(GOLD, "single_particle_cic.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            c, z, y, x, val = line.split()
            want["xyz".index(c), int(z), int(y), int(x)] = float(Fraction(val))
    np.testing.assert_allclose(np.stack(J), want, rtol=0, atol=1e-15)


def test_single_particle_order3_on_node():
    """Particle exactly on node (5, 5, 5): nodal factors (1/6, 2/3, 1/6, 0), staggered
    factors (1/48, 23/48, 23/48, 1/48) starting one node lower."""
    g = OracleGrid(3, (10, 10, 10), order=3)
    pos = [np.array([5.0]), np.array([5.0]), np.array([5.0])]
    u = [np.array([0.0], np.float32), np.array([0.0], np.float32), np.array([0.75], np.float32)]
    w = np.array([1.0], np.float32)
    J = od.deposit(g, pos, u, w)
    nod = np.array([1 / 6, 2 / 3, 1 / 6])            # nodes 4, 5, 6 (node 7 has 0)
    stg = np.array([1, 23, 23, 1]) / 48.0            # nodes 3, 4, 5, 6
    qv = -1.0 * 0.6
    want = np.zeros(g.shape)
    want[3:7, 4:7, 4:7] = qv * stg[:, None, None] * nod[None, :, None] * nod[None, None, :]
    np.testing.assert_allclose(J[2], want, rtol=0, atol=1e-15)
    assert not J[0].any() and not J[1].any()


@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("bc", [PERIODIC, GUARD])
@pytest.mark.parametrize("dim", [2, 3])
def test_bruteforce_equals_stencil(order, bc, dim):
    n = (6, 5, 7)[:dim] if bc == PERIODIC else (5, 4, 6)[:dim]
    g = OracleGrid(dim, n, order, q=-1.0, bc=(bc,) * 3, ng=3 if bc == GUARD else 0)
    pos, u, w = _rand_particles(g, 25, seed=order * 10 + dim)
    Js = od.deposit(g, pos, u, w)
    Jb = od.deposit_bruteforce(g, pos, u, w)
    for a, b in zip(Js, Jb):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)


@pytest.mark.parametrize("order", [1, 3])
def test_add_at_equals_bincount(order):
    g = OracleGrid(3, (5, 5, 6), order)
    pos, u, w = _rand_particles(g, 15, seed=5)
    for a, b in zip(od.deposit(g, pos, u, w), od.deposit_add_at(g, pos, u, w)):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)


@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("bc", [PERIODIC, GUARD])
def test_partition_of_unity(order, bc):
    g = OracleGrid(3, (8, 7, 9), order, q=-1.0, bc=(bc,) * 3, ng=3)
    pos, u, w = _rand_particles(g, 3000, seed=21)
    J = od.deposit(g, pos, u, w)
    _, v = od.velocity(u)
    for c in range(3):
        want = g.q * np.sum(w.astype(np.float64) * v[c])
        assert abs(J[c].sum() - want) <= 1e-13 * np.sum(np.abs(w * v[c]))


@pytest.mark.parametrize("order", [1, 2, 3])
def test_first_moment_guard(order):
    """sum_m X_c(m) J_c(m) = q sum_p w v_c x_p with X the (staggered) node position."""
    g = OracleGrid(3, (6, 7, 5), order, q=-1.0, bc=(GUARD,) * 3, ng=3)
    pos, u, w = _rand_particles(g, 2000, seed=8)
    J = od.deposit(g, pos, u, w)
    _, v = od.velocity(u)
    for c in range(3):
        for d in range(3):
            coords = np.arange(-g.ng, g.n[d] + g.ng) + od.stagger(g, c, d)
            shape = [1, 1, 1]
            shape[2 - d] = -1
            lhs = (J[c] * coords.reshape(shape)).sum()
            rhs = g.q * np.sum(w * v[c] * pos[d])
            assert abs(lhs - rhs) <= 1e-11 * np.sum(np.abs(w * v[c] * pos[d])) + 1e-12


@pytest.mark.parametrize("order", [1, 2, 3])
def test_uniform_lattice_is_constant(order):
    """One particle per cell at the same offset and velocity: J_c = q w v_c everywhere."""
    g = OracleGrid(3, (6, 5, 4), order)
    k, j, i = np.meshgrid(np.arange(4), np.arange(5), np.arange(6), indexing="ij")
    off = (0.3, 0.71, 0.5)
    pos = [i.ravel() + off[0], j.ravel() + off[1], k.ravel() + off[2]]
    N = i.size
    u = [np.full(N, 0.2, np.float32), np.full(N, -0.1, np.float32), np.full(N, 0.05, np.float32)]
    w = np.full(N, 1.5, np.float32)
    J = od.deposit(g, pos, u, w)
    _, v = od.velocity([a[:1] for a in u])
    for c in range(3):
        np.testing.assert_allclose(J[c], g.q * 1.5 * v[c][0], rtol=1e-14)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_integer_translation_rolls(order):
    g = OracleGrid(3, (7, 6, 5), order)
    pos, u, w = _rand_particles(g, 400, seed=2)
    pos = [np.round(p * 2.0 ** 20) / 2.0 ** 20 for p in pos]   # integer shifts stay exact
    J = od.deposit(g, pos, u, w)
    shift = (2, 3, 1)
    moved = [np.mod(pos[d] + shift[d], g.n[d]) for d in range(3)]
    J2 = od.deposit(g, moved, u, w)
    for c in range(3):
        np.testing.assert_array_equal(J2[c], np.roll(J[c], shift[::-1], axis=(0, 1, 2)))


def test_linearity():
    g = OracleGrid(3, (6, 6, 6), 3)
    pos, u, w = _rand_particles(g, 300, seed=4)
    sel = np.zeros(300, bool)
    sel[::3] = True
    JA = od.deposit(g, pos, u, w, valid=sel)
    JB = od.deposit(g, pos, u, w, valid=~sel)
    J = od.deposit(g, pos, u, w)
    for c in range(3):
        np.testing.assert_allclose(J[c], JA[c] + JB[c], rtol=0, atol=1e-13)


def test_upper_boundary_clamp_and_errors():
    g = OracleGrid(3, (4, 4, 4), 1, bc=(GUARD,) * 3, ng=1)
    pos = [np.array([4.0]), np.array([1.5]), np.array([2.5])]
    u = [np.array([0.1], np.float32)] * 3
    w = np.array([1.0], np.float32)
    J = od.deposit(g, pos, u, w)          # on the upper face: allowed (clamped cell)
    _, cells = od.grid_coords(g, pos)
    assert int(cells[0][0]) == 3
    assert np.isfinite(J[0]).all()
    with pytest.raises(od.OutOfDomain):
        od.deposit(g, [np.array([4.5]), pos[1], pos[2]], u, w)
    with pytest.raises(od.OutOfDomain):
        od.deposit(g, [np.array([-0.25]), pos[1], pos[2]], u, w)
    # only xi == n itself is clamped: half a cell beyond the face is outside even where
    # the stencil would wrap (periodic) and hide it
    gp = OracleGrid(3, (4, 4, 4), 1)
    with pytest.raises(od.OutOfDomain):
        od.grid_coords(gp, [np.array([4.5]), np.array([1.0]), np.array([1.0])])
    _, cells = od.grid_coords(gp, [np.array([4.0]), np.array([1.0]), np.array([1.0])])
    assert int(cells[0][0]) == 3


def test_2d_c1_shape_partition():
    params, arr = synth.uniform(2, (16, 16), 4, 0.01, 1, seed=9)
    g = OracleGrid.from_params(params)
    pos = [arr["x"], arr["y"], arr["z"]]
    u = [arr["ux"], arr["uy"], arr["uz"]]
    J = od.deposit(g, pos, u, arr["w"])
    assert J[0].shape == (16, 16)
    _, v = od.velocity(u)
    for c in range(3):
        assert abs(J[c].sum() - g.q * np.sum(arr["w"] * v[c])) < 1e-12


def test_planted_missing_stagger_is_caught(monkeypatch):
    """Depositing Jx on nodes instead of half nodes breaks the first-moment pin."""
    g = OracleGrid(3, (6, 7, 5), 3, bc=(GUARD,) * 3, ng=3)
    pos, u, w = _rand_particles(g, 500, seed=8)
    monkeypatch.setattr(od, "stagger", lambda g_, c, d: 0.0)
    J = od.deposit(g, pos, u, w)
    monkeypatch.undo()
    _, v = od.velocity(u)
    coords = np.arange(-g.ng, g.n[0] + g.ng) + 0.5
    lhs = (J[0] * coords.reshape(1, 1, -1)).sum()
    rhs = g.q * np.sum(w * v[0] * pos[0])
    assert abs(lhs - rhs) > 1e-3 * abs(rhs)
