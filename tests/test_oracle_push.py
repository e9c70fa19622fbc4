"""Pins of the Boris-push oracle: field-free drift, pure electric kick, pure magnetic
rotation (|u| kept, angle 2 atan(|t|)), and momentum parallel to B left alone."""
import numpy as np
import pytest

from oracle import deposit as od
from oracle.deposit import OracleGrid


def _setup(seed, N=50):
    g = OracleGrid(3, (8, 7, 6), 3)
    rng = np.random.default_rng(seed)
    pos = [rng.uniform(0, g.n[d], N) for d in range(3)]
    u = [rng.normal(0, 0.3, N).astype(np.float32) for _ in range(3)]
    return g, pos, u


def _const(g, v):
    return [np.full(g.shape, c) for c in v]


def test_no_field_is_drift():
    g, pos, u = _setup(1)
    p2, u2 = od.boris_push(g, pos, u, _const(g, (0, 0, 0)), _const(g, (0, 0, 0)), -1.0, 0.3)
    for c in range(3):
        assert np.array_equal(u2[c], u[c])
    d = od.drift(g, pos, u, 0.3)
    for k in range(3):
        assert np.array_equal(p2[k], d[k])


def test_pure_electric_kick():
    g, pos, u = _setup(2)
    Ev = (0.2, -0.1, 0.05)
    _, u2 = od.boris_push(g, pos, u, _const(g, Ev), _const(g, (0, 0, 0)), -2.0, 0.5)
    for c in range(3):
        want = (np.float64(1) * u[c] + (-2.0) * 0.5 * Ev[c]).astype(np.float32)
        np.testing.assert_allclose(u2[c], want, rtol=0, atol=2e-7)


def test_pure_magnetic_rotation():
    g, pos, u = _setup(3)
    Bz = 0.7
    qm, dt = -1.0, 0.4
    _, u2 = od.boris_push(g, pos, u, _const(g, (0, 0, 0)), _const(g, (0, 0, Bz)), qm, dt)
    u64 = [np.asarray(c, np.float64) for c in u]
    gam = np.sqrt(1 + u64[0] ** 2 + u64[1] ** 2 + u64[2] ** 2)
    n0 = np.hypot(u64[0], u64[1])
    n1 = np.hypot(u2[0].astype(np.float64), u2[1].astype(np.float64))
    np.testing.assert_allclose(n1, n0, rtol=1e-6)                 # |u_perp| kept
    np.testing.assert_array_equal(u2[2], u[2])                   # u_par untouched
    ang0 = np.arctan2(u64[1], u64[0])
    ang1 = np.arctan2(u2[1].astype(np.float64), u2[0].astype(np.float64))
    rot = np.angle(np.exp(1j * (ang1 - ang0)))
    tmag = 0.5 * qm * dt * Bz / gam
    np.testing.assert_allclose(rot, -2.0 * np.arctan(tmag), rtol=0, atol=1e-6)


def _parts(g, seed, N=60, sig=0.5):
    rng = np.random.default_rng(seed)
    pos = [rng.uniform(0, g.n[d], N) for d in range(g.dim)]
    u = [rng.normal(0, sig, N).astype(np.float32) for _ in range(3)]
    w = rng.uniform(0.5, 1.5, N)
    return pos, u, w


@pytest.mark.parametrize("order", [1, 2, 3])
def test_midpoint_both_ends_agree(order):
    """Depositing from the start of the move (+dt/2) and from its end (-dt/2) gives the
    same current: a sign error in either form breaks this."""
    g = OracleGrid(3, (9, 8, 7), order)
    pos, u, w = _parts(g, 10 + order)
    dt = 0.7
    end = od.drift(g, pos, u, dt)
    a = od.deposit_midpoint(g, pos, u, w, dt, moved=False)
    b = od.deposit_midpoint(g, end, u, w, dt, moved=True)
    for c in range(3):
        np.testing.assert_allclose(a[c], b[c], rtol=0, atol=1e-9 * np.abs(a[c]).max())


def test_midpoint_at_rest_is_plain_deposit():
    g = OracleGrid(2, (12, 10), 2)
    pos, u, w = _parts(g, 21)
    zero = [np.zeros_like(c) for c in u]
    a = od.deposit_midpoint(g, pos, zero, w, 0.9, moved=True)
    b = od.deposit(g, pos, zero, w)
    for c in range(3):
        assert np.array_equal(a[c], b[c])


def test_midpoint_single_particle_cic_weights():
    """One particle, order 1: Jx at the midpoint has the hand-computed CIC weights."""
    g = OracleGrid(3, (6, 6, 6), 1)
    ux = np.float32(0.75)                 # gamma = 1.25, vx = 0.6
    pos = [np.array([2.3]), np.array([3.0]), np.array([1.0])]
    u = [np.array([ux]), np.zeros(1, np.float32), np.zeros(1, np.float32)]
    J = od.deposit_midpoint(g, pos, u, np.array([1.0]), 1.0, moved=True)
    # midpoint x = 2.3 - 0.3 = 2.0; Jx is staggered by 1/2: nodes 1.5 and 2.5 share it
    jx = J[0][1, 3, :]
    q = g.q * 0.6
    np.testing.assert_allclose(jx[1], 0.5 * q, rtol=1e-12)
    np.testing.assert_allclose(jx[2], 0.5 * q, rtol=1e-12)
    assert np.isclose(np.abs(J[0]).sum(), abs(q), rtol=1e-12)
