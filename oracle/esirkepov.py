"""Charge-conserving current deposition (Esirkepov's density decomposition), FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper deposits the direct current of Eq. 1 and names charge-conserving schemes
(Esirkepov / Vay) as not supported (Sec. 7, limitations). This oracle follows the
published method: T. Zh. Esirkepov, "Exact charge conservation scheme for
Particle-in-Cell simulation with an arbitrary form-factor", Comput. Phys. Commun. 135
(2001) 144. For a particle that moves from grid coordinate xi0 to xi1 in one step
(|xi1 - xi0| < 1 cell per dimension), with 1D nodal weights S0_d(m) = B_o(m - xi0_d),
S1_d(m) = B_o(m - xi1_d) and DS = S1 - S0 on a common box of o+2 nodes per dimension,

  3D:  W_x(i,j,k) = DSx_i (S0y_j S0z_k + 1/2 DSy_j S0z_k + 1/2 S0y_j DSz_k + 1/3 DSy_j DSz_k)
       (W_y, W_z by cyclic exchange), and the current on the half-integer x faces
       Jx(i+1/2, j, k) = -q W dx/dt sum_{i' <= i} W_x(i', j, k);
  2D:  W_x(i,j) = DSx_i (S0y_j + 1/2 DSy_j), W_y likewise, and the out-of-plane current
       Jz(i,j) = q W v_z (S0x S0y + 1/2 DSx S0y + 1/2 S0x DSy + 1/3 DSx DSy) at the nodes.

Sum_d W_d = S1 S1 (S1) - S0 S0 (S0), which makes the discrete continuity equation
(rho1 - rho0)/dt + div J = 0 hold exactly with the nodal charge density of the same order.

Readings: J_d at storage index i is the face value at i + 1/2 (the Yee staggering of Eq. 1's
J); no 1/cell-volume factor (as Eq. 1); periodic displacements take the nearest image;
a move of a whole cell or more along any dimension is an error (the box would not hold
both stencils). All arithmetic float64, one particle's box at a time, vectorised over
particles.
"""
import numpy as np

from . import shapes
from .deposit import PERIODIC, _flat, _node_index, _select, grid_coords, velocity


class MoveTooLarge(ValueError):
    pass


def _boxes(g, xi0, xi1):
    """Per dimension: box node indices m (P, o+2) and the weights S0, S1 on them."""
    o = g.order
    out = []
    for d in range(g.dim):
        a = xi0[d]
        step = xi1[d] - xi0[d]
        if g.bc[d] == PERIODIC:
            step = step - g.n[d] * np.round(step / g.n[d])
        if np.any(np.abs(step) >= 1.0):
            raise MoveTooLarge(f"a particle moved a cell or more along dimension {d}")
        b = a + step
        first = np.floor(np.minimum(a, b) - 0.5 * (o + 1)).astype(np.int64) + 1
        m = first[:, None] + np.arange(o + 2)[None, :]
        s0 = shapes.kernel(o, m - a[:, None])
        s1 = shapes.kernel(o, m - b[:, None])
        out.append((m, s0, s1))
    return out


def deposit_esirkepov(g, pos_old, pos_new, u, w, dt, valid=None):
    """[Jx, Jy, Jz] (each g.shape) of the particles moving pos_old -> pos_new in dt."""
    pos_old = _select(pos_old[: g.dim], valid)
    pos_new = _select(pos_new[: g.dim], valid)
    u = _select(u, valid)
    w = _select([w], valid)[0].astype(np.float64)
    xi0, _ = grid_coords(g, pos_old)
    xi1, _ = grid_coords(g, pos_new)
    box = _boxes(g, xi0, xi1)
    qw = g.q * w
    P = qw.size
    if g.dim == 3:
        (mx, s0x, s1x), (my, s0y, s1y), (mz, s0z, s1z) = box
        dsx, dsy, dsz = s1x - s0x, s1y - s0y, s1z - s0z
        e = lambda a, b, c: a[:, :, None, None] * b[:, None, :, None] * c[:, None, None, :]
        Wx = (e(dsx, s0y, s0z) + 0.5 * e(dsx, dsy, s0z) + 0.5 * e(dsx, s0y, dsz)
              + (1.0 / 3.0) * e(dsx, dsy, dsz))
        Wy = (e(s0x, dsy, s0z) + 0.5 * e(dsx, dsy, s0z) + 0.5 * e(s0x, dsy, dsz)
              + (1.0 / 3.0) * e(dsx, dsy, dsz))
        Wz = (e(s0x, s0y, dsz) + 0.5 * e(dsx, s0y, dsz) + 0.5 * e(s0x, dsy, dsz)
              + (1.0 / 3.0) * e(dsx, dsy, dsz))
        vals = []
        for d, W in enumerate((Wx, Wy, Wz)):
            c = -np.cumsum(W, axis=1 + d) * (qw * g.dx[d] / dt)[:, None, None, None]
            vals.append(c)
    else:
        (mx, s0x, s1x), (my, s0y, s1y) = box
        dsx, dsy = s1x - s0x, s1y - s0y
        e = lambda a, b: a[:, :, None] * b[:, None, :]
        Wx = e(dsx, s0y) + 0.5 * e(dsx, dsy)
        Wy = e(s0x, dsy) + 0.5 * e(dsx, dsy)
        _, v = velocity(u)
        Jz = (e(s0x, s0y) + 0.5 * e(dsx, s0y) + 0.5 * e(s0x, dsy)
              + (1.0 / 3.0) * e(dsx, dsy)) * (qw * v[2])[:, None, None]
        vals = [-np.cumsum(Wx, axis=1) * (qw * g.dx[0] / dt)[:, None, None],
                -np.cumsum(Wy, axis=2) * (qw * g.dx[1] / dt)[:, None, None], Jz]
    nodes = [b[0] for b in box]
    J = []
    for c in range(3):
        val = vals[c].reshape(P, -1)
        grids = np.meshgrid(*[np.arange(g.order + 2)] * g.dim, indexing="ij")
        idx = []
        for d in range(g.dim):
            m = nodes[d][:, grids[d].reshape(-1)]
            idx.append(_node_index(g, d, m, val))
        flat = _flat(g, idx).reshape(-1)
        J.append(np.bincount(flat, weights=val.reshape(-1), minlength=g.size).reshape(g.shape))
    return J
