"""1D shape factors (B-splines) used by the deposition oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper writes the 3D shape as a product of 1D factors, S_ijk = s_x,i * s_y,j * s_z,k
(Sec. 4.2.1, the equation for rhocell updates and the text after it), gives the
first-order (CIC) factors explicitly as s0 = 1 - dx, s1 = dx (Sec. 4.2.2, Stage 1), and
names second order (TSC) and third order ("QSP", four terms per dimension) as the
higher-order schemes (Sec. 4.2.1, last paragraph). The textbook definition it relies on
(Hockney & Eastwood, cited in Sec. 3.1) is the cardinal B-spline of degree `order`:

    B_1(t) = max(0, 1 - |t|)
    B_2(t) = 3/4 - t^2                  for |t| <= 1/2
           = (3/2 - |t|)^2 / 2          for 1/2 < |t| <= 3/2, else 0
    B_3(t) = 2/3 - t^2 + |t|^3 / 2      for |t| <= 1
           = (2 - |t|)^3 / 6            for 1 < |t| <= 2, else 0

and a particle at grid coordinate xi gives node m the weight B_o(m - xi).

`weights(order, xi)` returns the order+1 non-zero weights and the first node index
(`base`); `dweights` returns d/dxi of the same weights. Reading (the paper does not
state it): the stencil for a particle at xi starts at
    order 1: floor(xi),  order 2: floor(xi + 1/2) - 1,  order 3: floor(xi) - 1.
All arithmetic is float64.
"""
import numpy as np

ORDERS = (1, 2, 3)


def kernel(order, t):
    """Continuous cardinal B-spline B_order(t) (definition above)."""
    a = np.abs(np.asarray(t, dtype=np.float64))
    if order == 1:
        return np.maximum(0.0, 1.0 - a)
    if order == 2:
        inner = 0.75 - a * a
        outer = 0.5 * (1.5 - a) ** 2
        return np.where(a <= 0.5, inner, np.where(a <= 1.5, outer, 0.0))
    if order == 3:
        inner = 2.0 / 3.0 - a * a + 0.5 * a ** 3
        outer = (2.0 - a) ** 3 / 6.0
        return np.where(a <= 1.0, inner, np.where(a <= 2.0, outer, 0.0))
    raise ValueError(f"order must be 1, 2 or 3, got {order}")


def dkernel(order, t):
    """d B_order(t) / dt (one-sided values at the kinks of orders 1 and 2 are not used)."""
    t = np.asarray(t, dtype=np.float64)
    a = np.abs(t)
    s = np.sign(t)
    if order == 1:
        return np.where(a < 1.0, -s, 0.0)
    if order == 2:
        return np.where(a <= 0.5, -2.0 * t, np.where(a <= 1.5, -s * (1.5 - a), 0.0))
    if order == 3:
        inner = s * (-2.0 * a + 1.5 * a * a)
        outer = -s * 0.5 * (2.0 - a) ** 2
        return np.where(a <= 1.0, inner, np.where(a <= 2.0, outer, 0.0))
    raise ValueError(f"order must be 1, 2 or 3, got {order}")


def _frac(order, xi):
    """First stencil node and the local coordinate the weight polynomials use."""
    xi = np.asarray(xi, dtype=np.float64)
    if order == 1:
        fl = np.floor(xi)
        return fl.astype(np.int64), xi - fl
    if order == 2:
        r = np.floor(xi + 0.5)
        return (r - 1).astype(np.int64), xi - r          # g in [-1/2, 1/2)
    if order == 3:
        fl = np.floor(xi)
        return (fl - 1).astype(np.int64), xi - fl         # f in [0, 1)
    raise ValueError(f"order must be 1, 2 or 3, got {order}")


def weights(order, xi):
    """Return (base, W) with W[..., k] = B_order(base + k - xi), k = 0..order.

    Closed forms (polynomial pieces of B_order on the stencil):
      order 1, f = xi - floor(xi):          [1 - f, f]
      order 2, g = xi - floor(xi + 1/2):    [(1/2 - g)^2 / 2, 3/4 - g^2, (1/2 + g)^2 / 2]
      order 3, f = xi - floor(xi):          [(1-f)^3/6, (4 - 6f^2 + 3f^3)/6,
                                             (1 + 3f + 3f^2 - 3f^3)/6, f^3/6]
    """
    base, f = _frac(order, xi)
    if order == 1:
        W = np.stack([1.0 - f, f], axis=-1)
    elif order == 2:
        W = np.stack([0.5 * (0.5 - f) ** 2, 0.75 - f * f, 0.5 * (0.5 + f) ** 2], axis=-1)
    else:
        f2 = f * f
        f3 = f2 * f
        W = np.stack([(1.0 - f) ** 3 / 6.0,
                      (4.0 - 6.0 * f2 + 3.0 * f3) / 6.0,
                      (1.0 + 3.0 * f + 3.0 * f2 - 3.0 * f3) / 6.0,
                      f3 / 6.0], axis=-1)
    return base, W


def dweights(order, xi):
    """Return (base, dW) with dW[..., k] = d/dxi B_order(base + k - xi)."""
    base, f = _frac(order, xi)
    if order == 1:
        one = np.ones_like(f)
        dW = np.stack([-one, one], axis=-1)
    elif order == 2:
        dW = np.stack([-(0.5 - f), -2.0 * f, 0.5 + f], axis=-1)
    else:
        dW = np.stack([-0.5 * (1.0 - f) ** 2,
                       -2.0 * f + 1.5 * f * f,
                       0.5 + f - 1.5 * f * f,
                       0.5 * f * f], axis=-1)
    return base, dW
