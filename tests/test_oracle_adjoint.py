"""Pins of the adjoint oracle: exact identities and float64 central differences."""
import numpy as np
import pytest

from oracle import deposit as od
from oracle.deposit import GUARD, PERIODIC, OracleGrid


def _setup(order, bc=PERIODIC, N=200, seed=0, dim=3):
    n = (7, 6, 8)[:dim]
    g = OracleGrid(dim, n, order, q=-1.0, bc=(bc,) * 3, ng=3)
    rng = np.random.default_rng(seed)
    pos = [rng.uniform(0, g.n[d], N) for d in range(dim)] + [np.zeros(N)] * (3 - dim)
    u = [rng.normal(0, 0.4, N).astype(np.float32) for _ in range(3)]
    w = rng.uniform(0.5, 2, N).astype(np.float32)
    G = [rng.normal(0, 1, g.shape) for _ in range(3)]
    return g, pos, u, w, G


def _loss_one(g, pos, u, w, G, p, which=None, h=0.0):
    """L_p = sum_c <G_c, J_c^(p)> for particle p with one input perturbed (float64)."""
    P = [np.array([float(pos[d][p])]) for d in range(3)]
    U = [np.array([float(u[c][p])]) for c in range(3)]
    W = np.array([float(w[p])])
    if which is not None:
        kind, k = which
        {"x": P, "u": U}[kind][k][0] += h
    # promote: feed float64 u and w directly (the oracle casts to float64 anyway)
    J = od.deposit(g, P, U, W)
    return sum(float((J[c] * G[c]).sum()) for c in range(3))


@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("bc", [PERIODIC, GUARD])
def test_dot_product_identity(order, bc):
    """L is linear in w, so sum_c <G_c, J_c> = sum_p w_p dL/dw_p exactly."""
    g, pos, u, w, G = _setup(order, bc)
    J = od.deposit(g, pos, u, w)
    L = sum((J[c] * G[c]).sum() for c in range(3))
    grads = od.deposit_adjoint(g, pos, u, w, G)
    assert abs(L - np.sum(w * grads["dw"])) <= 1e-12 * max(1.0, abs(L))


@pytest.mark.parametrize("order", [1, 2, 3])
def test_constant_field(order):
    """Constant G: dL/dx = 0 (weights sum to one) and dL/du = q w G . dv/du in closed form."""
    g, pos, u, w, _ = _setup(order)
    Gc = (0.7, -1.3, 2.1)
    G = [np.full(g.shape, v) for v in Gc]
    out = od.deposit_adjoint(g, pos, u, w, G)
    for name in ("dx", "dy", "dz"):
        np.testing.assert_allclose(out[name], 0.0, atol=1e-12)
    uu = [np.asarray(c, np.float64) for c in u]
    gam = np.sqrt(1 + uu[0] ** 2 + uu[1] ** 2 + uu[2] ** 2)
    for b, name in enumerate(("dux", "duy", "duz")):
        want = np.zeros_like(gam)
        for c in range(3):
            want += Gc[c] * ((c == b) / gam - uu[c] * uu[b] / gam ** 3)
        np.testing.assert_allclose(out[name], g.q * w * want, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("bc", [PERIODIC, GUARD])
@pytest.mark.parametrize("dim", [2, 3])
def test_central_differences(order, bc, dim):
    g, pos, u, w, G = _setup(order, bc, N=60, seed=order + 5 * dim, dim=dim)
    out = od.deposit_adjoint(g, pos, u, w, G)
    h = 1e-6
    for p in range(60):
        for d in range(dim):
            xi = pos[d][p]
            # kinks of orders 1 and 2 (integer / half-integer points of xi and xi - 1/2)
            if order < 3:
                frac = (xi - np.floor(xi)) % 0.5
                if min(frac, 0.5 - frac) < 4 * h:
                    continue
            fd = (_loss_one(g, pos, u, w, G, p, ("x", d), h)
                  - _loss_one(g, pos, u, w, G, p, ("x", d), -h)) / (2 * h)
            assert abs(out[("dx", "dy", "dz")[d]][p] - fd) <= 1e-6 * max(1.0, abs(fd))
        for b in range(3):
            fd = (_loss_one(g, pos, u, w, G, p, ("u", b), h)
                  - _loss_one(g, pos, u, w, G, p, ("u", b), -h)) / (2 * h)
            assert abs(out[("dux", "duy", "duz")[b]][p] - fd) <= 1e-7 * max(1.0, abs(fd))


def test_planted_sign_slip_is_caught():
    """Flipping the u_c u_b / gamma^3 sign breaks the constant-field closed form."""
    g, pos, u, w, _ = _setup(3)
    Gc = (0.7, -1.3, 2.1)
    G = [np.full(g.shape, v) for v in Gc]
    out = od.deposit_adjoint(g, pos, u, w, G)
    uu = [np.asarray(c, np.float64) for c in u]
    gam = np.sqrt(1 + uu[0] ** 2 + uu[1] ** 2 + uu[2] ** 2)
    wrong = sum(Gc[c] * ((c == 0) / gam + uu[c] * uu[0] / gam ** 3) for c in range(3))
    assert np.max(np.abs(out["dux"] - g.q * w * wrong)) > 1e-3
