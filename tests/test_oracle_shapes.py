"""Pins of the oracle's 1D shape factors against values the mathematics fixes."""
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import shapes

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden_weights():
    rows = []
    with open(os.path.join(GOLD, "bspline_weights.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            rows.append((int(t[0]), float(t[1]), int(t[2]), [float(Fraction(v)) for v in t[3:]]))
    return rows


@pytest.mark.parametrize("row", _golden_weights())
def test_golden_closed_forms(row):
    order, xi, base, want = row
    b, W = shapes.weights(order, np.array([xi]))
    assert int(b[0]) == base
    np.testing.assert_allclose(W[0], want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("order", shapes.ORDERS)
def test_against_scipy_bspline_basis(order):
    """Cardinal B-spline of degree `order` = scipy's basis element on centred integer knots."""
    knots = np.arange(order + 2) - (order + 1) / 2.0
    ref = BSpline.basis_element(knots, extrapolate=False)
    t = np.linspace(-3, 3, 1201)
    want = np.nan_to_num(ref(t))
    np.testing.assert_allclose(shapes.kernel(order, t), want, rtol=0, atol=1e-14)


@pytest.mark.parametrize("order", shapes.ORDERS)
def test_stencil_equals_kernel(order):
    rng = np.random.default_rng(7)
    xi = rng.uniform(-5, 50, 4000)
    base, W = shapes.weights(order, xi)
    m = base[:, None] + np.arange(order + 1)[None, :]
    np.testing.assert_allclose(W, shapes.kernel(order, m - xi[:, None]), rtol=0, atol=2e-15)
    # nodes just outside the stencil carry no weight
    assert np.all(shapes.kernel(order, (base - 1) - xi) < 1e-15)
    assert np.all(shapes.kernel(order, (base + order + 1) - xi) < 1e-15)


@pytest.mark.parametrize("order", shapes.ORDERS)
def test_moments(order):
    """Partition of unity, first moment = xi, second moment = (o+1)/12 (f(1-f) for o=1)."""
    rng = np.random.default_rng(11)
    xi = rng.uniform(0, 100, 5000)
    base, W = shapes.weights(order, xi)
    m = base[:, None] + np.arange(order + 1)[None, :]
    np.testing.assert_allclose(W.sum(1), 1.0, rtol=0, atol=1e-14)
    np.testing.assert_allclose((m * W).sum(1), xi, rtol=1e-14, atol=1e-12)
    var = ((m - xi[:, None]) ** 2 * W).sum(1)
    if order == 1:
        f = xi - np.floor(xi)
        np.testing.assert_allclose(var, f * (1 - f), rtol=0, atol=1e-12)
    else:
        np.testing.assert_allclose(var, (order + 1) / 12.0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("order", shapes.ORDERS)
def test_derivative_weights_central_difference(order):
    rng = np.random.default_rng(3)
    xi = rng.uniform(0, 20, 2000)
    h = 1e-6
    base, dW = shapes.dweights(order, xi)
    m = base[:, None] + np.arange(order + 1)[None, :]
    fd = (shapes.kernel(order, m - (xi[:, None] + h)) - shapes.kernel(order, m - (xi[:, None] - h))) / (2 * h)
    # orders 1 and 2 have kinks: skip points within 2h of one
    if order == 1:
        ok = np.abs(xi - np.round(xi)) > 2 * h
    elif order == 2:
        ok = np.abs((xi - 0.5) - np.round(xi - 0.5)) > 2 * h
    else:
        ok = np.ones_like(xi, dtype=bool)
    np.testing.assert_allclose(dW[ok], fd[ok], rtol=0, atol=2e-8)
    np.testing.assert_allclose(dW.sum(1), 0.0, atol=1e-13)
    np.testing.assert_allclose(shapes.dkernel(order, (m - xi[:, None])[ok]) * -1, dW[ok], atol=1e-13)


def test_planted_wrong_cubic_piece_is_caught(monkeypatch):
    """A plausible slip (1 + 3f + 3f^2 - 3f^3 written with +3f^3) breaks the pins."""
    real = shapes.weights

    def wrong(order, xi):
        base, W = real(order, xi)
        if order == 3:
            f = np.asarray(xi) - np.floor(xi)
            W = W.copy()
            W[..., 2] = (1 + 3 * f + 3 * f * f + 3 * f ** 3) / 6
        return base, W

    monkeypatch.setattr(shapes, "weights", wrong)
    xi = np.array([5.25])
    _, W = shapes.weights(3, xi)
    assert abs(W.sum() - 1.0) > 1e-3
