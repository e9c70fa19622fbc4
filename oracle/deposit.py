"""Direct FP64 evaluation of current deposition, its adjoint, and the drift between steps.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

What is computed (Sec. 3.1, Eq. 1; Sec. 4.2.1, the rhocell update equation with
w_p = q_p v_p W_p):

    J_c(node m) = sum_p  q * W_p * v_{p,c} * prod_d  B_o(m_d + sigma_{c,d} - xi_{p,d})

Readings where the paper is silent (each is listed in the design notes):
  * Yee staggering: component c sits half a cell along its own axis, sigma_{c,d} = 1/2
    if d == c else 0. In 2D (x, y) Jz has sigma = 0 in both dimensions.
  * Grid coordinate: xi_d = (x_d - x0_d) * inv_dx_d, two separately rounded float64
    operations. Cell i_d = floor(xi_d); xi_d == n_d is clamped into cell n_d - 1.
    Any other cell outside [0, n_d) is an error.
  * Momenta are proper velocities u (c = 1): gamma = sqrt(1 + |u|^2), v = u / gamma.
  * No 1/cell-volume normalisation (Eq. 1 has none).
  * Boundaries per dimension: periodic (node m wraps mod n_d) or guard (node m is
    stored at m + ng; it is an error if m + ng falls outside [0, n_d + 2 ng)).
  * Layout of every grid array: x fastest, shape (Nz, Ny, Nx) in 3D and (Ny, Nx) in
    2D, N_d = n_d + 2 ng on guard dimensions and n_d on periodic ones.
The scatter is a plain np.bincount per stencil node; nothing is blocked or fused.
"""
import numpy as np

from . import shapes

PERIODIC = 0
GUARD = 1


class OracleGrid:
    """Grid descriptor as the oracle reads it (independent of the library's struct)."""

    def __init__(self, dim, n, order, q=-1.0, x0=(0.0, 0.0, 0.0), dx=(1.0, 1.0, 1.0),
                 bc=(PERIODIC, PERIODIC, PERIODIC), ng=0):
        self.dim = int(dim)
        self.n = tuple(int(v) for v in n)[: self.dim]
        self.order = int(order)
        self.q = float(q)
        self.x0 = tuple(float(v) for v in x0)[: self.dim]
        self.dx = tuple(float(v) for v in dx)[: self.dim]
        self.inv_dx = tuple(1.0 / v for v in self.dx)
        self.bc = tuple(int(v) for v in bc)[: self.dim]
        self.ng = int(ng)

    @classmethod
    def from_params(cls, p):
        return cls(p["dim"], p["n"], p["order"], p["q"], p.get("x0", (0.0,) * 3),
                   p.get("dx", (1.0,) * 3), p.get("bc", (PERIODIC,) * 3), p.get("ng", 0))

    def guard(self, d):
        return self.ng if self.bc[d] == GUARD else 0

    @property
    def shape(self):
        """Array shape of one J component, slowest dimension first."""
        return tuple(self.n[d] + 2 * self.guard(d) for d in reversed(range(self.dim)))

    @property
    def size(self):
        return int(np.prod(self.shape))


class OutOfDomain(ValueError):
    pass


def grid_coords(g, pos):
    """Per dimension: xi_d (float64) and cell i_d (int64) with the boundary clamp."""
    xis, cells = [], []
    for d in range(g.dim):
        x = np.asarray(pos[d], dtype=np.float64)
        xi = (x - g.x0[d]) * g.inv_dx[d]
        i = np.floor(xi)
        i = np.where(xi == g.n[d], g.n[d] - 1, i)
        if np.any((i < 0) | (i >= g.n[d])):
            raise OutOfDomain(f"particle outside the domain along dimension {d}")
        xis.append(xi)
        cells.append(i.astype(np.int64))
    return xis, cells


def velocity(u):
    """gamma = sqrt(1 + ux^2 + uy^2 + uz^2), v = u / gamma, in float64."""
    ux, uy, uz = (np.asarray(c, dtype=np.float64) for c in u)
    gamma = np.sqrt(1.0 + (ux * ux + uy * uy + uz * uz))
    return gamma, (ux / gamma, uy / gamma, uz / gamma)


def stagger(g, comp, d):
    """sigma_{c,d}: half a cell along the component's own axis (Yee)."""
    return 0.5 if (comp == d and comp < g.dim) else 0.0


def _node_index(g, d, m, W):
    """Storage index along dimension d of node m (int64 array).

    On guard dimensions a node outside the stored range is an error unless its weight
    is exactly zero (the zero-weight end node of a particle sitting exactly on the
    upper domain boundary); such nodes are pointed at index 0 and add nothing.
    """
    if g.bc[d] == PERIODIC:
        return np.mod(m, g.n[d])
    idx = m + g.ng
    out = (idx < 0) | (idx >= g.n[d] + 2 * g.ng)
    if np.any(out & (W != 0.0)):
        raise OutOfDomain(f"stencil leaves the guard region along dimension {d}")
    return np.where(out, 0, idx)


def _flat(g, idx):
    """Flat x-fastest offset from per-dimension storage indices."""
    N = [g.n[d] + 2 * g.guard(d) for d in range(g.dim)]
    flat = idx[g.dim - 1]
    for d in reversed(range(g.dim - 1)):
        flat = flat * N[d] + idx[d]
    return flat


def _select(arrs, valid):
    if valid is None:
        return [np.asarray(a) for a in arrs]
    return [np.asarray(a)[valid] for a in arrs]


def _stencils(g, xis, comp, deriv_dim=None):
    """Per dimension: storage indices (P, o+1) and weights (P, o+1) for component comp.

    With deriv_dim = d, the weights along d are replaced by d/dxi_d of the weights.
    """
    out = []
    for d in range(g.dim):
        xs = xis[d] - stagger(g, comp, d)
        if deriv_dim == d:
            base, W = shapes.dweights(g.order, xs)
        else:
            base, W = shapes.weights(g.order, xs)
        m = base[:, None] + np.arange(g.order + 1)[None, :]
        out.append((_node_index(g, d, m, W), W))
    return out


def _combos(g):
    o1 = g.order + 1
    return np.array(np.meshgrid(*[np.arange(o1)] * g.dim, indexing="ij")).reshape(g.dim, -1).T


def deposit(g, pos, u, w, valid=None):
    """Eq. 1 with the readings above. Returns [Jx, Jy, Jz], each of shape g.shape."""
    pos = _select(pos[: g.dim], valid)
    u = _select(u, valid)
    w = _select([w], valid)[0].astype(np.float64)
    xis, _ = grid_coords(g, pos)
    _, v = velocity(u)
    J = []
    for comp in range(3):
        amp = g.q * w * v[comp]
        st = _stencils(g, xis, comp)
        acc = np.zeros(g.size, dtype=np.float64)
        for ks in _combos(g):
            val = amp.copy()
            idx = []
            for d in range(g.dim):
                val = val * st[d][1][:, ks[d]]
                idx.append(st[d][0][:, ks[d]])
            acc += np.bincount(_flat(g, idx), weights=val, minlength=g.size)
        J.append(acc.reshape(g.shape))
    return J


RHO = -1   # "component" of the charge density: nodal in every dimension


def deposit_rho(g, pos, w, valid=None):
    """Charge density, the scalar and nodal counterpart of Eq. 1 (the charge assignment of
    Appendix B): rho(m) = sum_p q W_p prod_d B_o(m_d - xi_{p,d}). Shape g.shape."""
    pos = _select(pos[: g.dim], valid)
    w = _select([w], valid)[0].astype(np.float64)
    xis, _ = grid_coords(g, pos)
    amp = g.q * w
    st = _stencils(g, xis, RHO)
    acc = np.zeros(g.size, dtype=np.float64)
    for ks in _combos(g):
        val = amp.copy()
        idx = []
        for d in range(g.dim):
            val = val * st[d][1][:, ks[d]]
            idx.append(st[d][0][:, ks[d]])
        acc += np.bincount(_flat(g, idx), weights=val, minlength=g.size)
    return acc.reshape(g.shape)


def deposit_rho_bruteforce(g, pos, w, valid=None):
    """All nodes x all particles with the continuous kernel B_o (tiny inputs only)."""
    pos = _select(pos[: g.dim], valid)
    w = _select([w], valid)[0].astype(np.float64)
    xis, _ = grid_coords(g, pos)
    prod = None
    for d in reversed(range(g.dim)):
        nodes = np.arange(-g.guard(d), g.n[d] + g.guard(d)).astype(np.float64)
        t = nodes[:, None] - xis[d][None, :]
        if g.bc[d] == PERIODIC:
            t = t - g.n[d] * np.round(t / g.n[d])
        k = shapes.kernel(g.order, t)
        prod = k if prod is None else (prod[:, None, :] * k[None, :, :]).reshape(-1, len(w))
    return (prod @ (g.q * w)).reshape(g.shape)


def deposit_add_at(g, pos, u, w, valid=None):
    """Same sum as deposit(), accumulated one particle and one node at a time.

    Independent of np.bincount; only for small inputs (pure Python loops).
    """
    pos = _select(pos[: g.dim], valid)
    u = _select(u, valid)
    w = _select([w], valid)[0].astype(np.float64)
    xis, _ = grid_coords(g, pos)
    _, v = velocity(u)
    J = [np.zeros(g.size) for _ in range(3)]
    combos = _combos(g)
    for comp in range(3):
        st = _stencils(g, xis, comp)
        for p in range(len(w)):
            amp = g.q * w[p] * v[comp][p]
            for ks in combos:
                val = amp
                idx = []
                for d in range(g.dim):
                    val *= st[d][1][p, ks[d]]
                    idx.append(np.array([st[d][0][p, ks[d]]]))
                J[comp][int(_flat(g, idx)[0])] += val
    return [a.reshape(g.shape) for a in J]


def deposit_bruteforce(g, pos, u, w, valid=None):
    """All nodes x all particles with the continuous kernel B_o (tiny inputs only).

    Periodic dimensions use the minimum image of (node - particle).
    """
    pos = _select(pos[: g.dim], valid)
    u = _select(u, valid)
    w = _select([w], valid)[0].astype(np.float64)
    xis, _ = grid_coords(g, pos)
    _, v = velocity(u)
    node_coords = []
    for d in range(g.dim):
        lo = -g.guard(d)
        node_coords.append(np.arange(lo, g.n[d] + g.guard(d)).astype(np.float64))
    J = []
    for comp in range(3):
        amp = g.q * w * v[comp]
        prod = None
        for d in reversed(range(g.dim)):
            t = node_coords[d][:, None] + stagger(g, comp, d) - xis[d][None, :]
            if g.bc[d] == PERIODIC:
                t = t - g.n[d] * np.round(t / g.n[d])
            k = shapes.kernel(g.order, t)                  # (N_d, P)
            prod = k if prod is None else prod[:, None, :] * k[None, :, :]
            prod = prod.reshape(-1, len(w))
        J.append((prod @ amp).reshape(g.shape))
    return J


def deposit_adjoint(g, pos, u, w, G, valid=None):
    """Adjoint of deposit() for L = sum_c <G_c, J_c>.

    Per particle p (gathered values g_c = sum_m G_c(m) S_c(m - x_p)):
      dL/dw     = q * sum_c v_c g_c
      dL/du_b   = q w sum_c (delta_cb / gamma - u_c u_b / gamma^3) g_c
      dL/dx_d   = q w sum_c v_c sum_m G_c(m) dS_c/dxi_d * inv_dx_d
    Returns a dict with keys dx, dy, dz (dz absent in 2D), dux, duy, duz, dw.
    """
    pos = _select(pos[: g.dim], valid)
    u = _select(u, valid)
    w = _select([w], valid)[0].astype(np.float64)
    xis, _ = grid_coords(g, pos)
    gamma, v = velocity(u)
    uu = [np.asarray(c, dtype=np.float64) for c in u]
    P = len(w)
    gath = []
    dgath = [[None] * g.dim for _ in range(3)]
    for comp in range(3):
        Gf = np.asarray(G[comp], dtype=np.float64).reshape(-1)
        st = _stencils(g, xis, comp)
        acc = np.zeros(P)
        for ks in _combos(g):
            idx = [st[d][0][:, ks[d]] for d in range(g.dim)]
            val = Gf[_flat(g, idx)]
            for d in range(g.dim):
                val = val * st[d][1][:, ks[d]]
            acc += val
        gath.append(acc)
        for dd in range(g.dim):
            std = _stencils(g, xis, comp, deriv_dim=dd)
            acc = np.zeros(P)
            for ks in _combos(g):
                idx = [std[d][0][:, ks[d]] for d in range(g.dim)]
                val = Gf[_flat(g, idx)]
                for d in range(g.dim):
                    val = val * std[d][1][:, ks[d]]
                acc += val
            dgath[comp][dd] = acc
    out = {"dw": g.q * sum(v[c] * gath[c] for c in range(3))}
    for b, name in enumerate(("dux", "duy", "duz")):
        tot = np.zeros(P)
        for c in range(3):
            dv = -uu[c] * uu[b] / gamma ** 3
            if c == b:
                dv = dv + 1.0 / gamma
            tot += dv * gath[c]
        out[name] = g.q * w * tot
    for d, name in enumerate(("dx", "dy", "dz")[: g.dim]):
        tot = sum(v[c] * dgath[c][d] for c in range(3))
        out[name] = g.q * w * tot * g.inv_dx[d]
    return out


def stagger_b(g, comp, d):
    """Magnetic component c sits half a cell along the two other axes (Yee faces)."""
    return 0.5 if (d != comp and d < g.dim) else 0.0


def _stencils_sigma(g, xis, sig):
    """Like _stencils for an explicit per-dimension shift sig[d] in {0, 1/2}."""
    out = []
    for d in range(g.dim):
        base, W = shapes.weights(g.order, xis[d] - sig[d])
        m = base[:, None] + np.arange(g.order + 1)[None, :]
        out.append((_node_index(g, d, m, W), W))
    return out


def _gather_one(g, F, xis, sig):
    Ff = np.asarray(F, dtype=np.float64).reshape(-1)
    st = _stencils_sigma(g, xis, sig)
    acc = np.zeros(len(xis[0]))
    for ks in _combos(g):
        idx = [st[d][0][:, ks[d]] for d in range(g.dim)]
        val = Ff[_flat(g, idx)]
        for d in range(g.dim):
            val = val * st[d][1][:, ks[d]]
        acc += val
    return acc


def gather_fields(g, pos, E, B, valid=None):
    """Field interpolation to the particles (the gather of Sec. 3.1, the forward of the
    adjoint's gather): E_c(x_p) = sum_m E_c(m) prod_d B_o(m_d + sigma^E_{c,d} - xi_{p,d}),
    likewise B_c with sigma^B. E_c sits on its own axis' edge (as J_c), B_c on the face
    normal to c (half a cell along the two other axes). Returns ([Ex, Ey, Ez], [Bx, By, Bz])
    per particle."""
    pos = _select(pos[: g.dim], valid)
    xis, _ = grid_coords(g, pos)
    Ep = [_gather_one(g, E[c], xis, [stagger(g, c, d) for d in range(g.dim)]) for c in range(3)]
    Bp = [_gather_one(g, B[c], xis, [stagger_b(g, c, d) for d in range(g.dim)]) for c in range(3)]
    return Ep, Bp


def gather_fields_bruteforce(g, pos, E, B, valid=None):
    """All nodes x all particles with the continuous kernel B_o (tiny inputs only)."""
    pos = _select(pos[: g.dim], valid)
    xis, _ = grid_coords(g, pos)

    def one(F, sig):
        prod = None
        for d in reversed(range(g.dim)):
            nodes = np.arange(-g.guard(d), g.n[d] + g.guard(d)).astype(np.float64)
            t = nodes[:, None] + sig[d] - xis[d][None, :]
            if g.bc[d] == PERIODIC:
                t = t - g.n[d] * np.round(t / g.n[d])
            k = shapes.kernel(g.order, t)
            prod = k if prod is None else (prod[:, None, :] * k[None, :, :]).reshape(-1, len(xis[0]))
        return np.asarray(F, dtype=np.float64).reshape(-1) @ prod

    Ep = [one(E[c], [stagger(g, c, d) for d in range(g.dim)]) for c in range(3)]
    Bp = [one(B[c], [stagger_b(g, c, d) for d in range(g.dim)]) for c in range(3)]
    return Ep, Bp


def drift(g, pos, u, dt):
    """Constant-velocity move x <- x + v dt between steps (float64), periodic wrap.

    Stand-in for the particle push, which the paper leaves to WarpX (Alg. 1). The
    order of operations is fixed so that an IEEE implementation reproduces it bit
    for bit: s = (ux*ux + uy*uy) + uz*uz, gamma = sqrt(1 + s), v_d = u_d / gamma,
    x_d + v_d * dt, then on periodic dimensions t = x - x0, t - L*floor(t / L), + x0.
    Guard dimensions are not wrapped.
    """
    ux, uy, uz = (np.asarray(c, dtype=np.float64) for c in u)
    s = (ux * ux + uy * uy) + uz * uz
    gamma = np.sqrt(1.0 + s)
    out = []
    for d in range(len(pos)):
        x = np.asarray(pos[d], dtype=np.float64)
        if d >= g.dim:
            out.append(x.copy())
            continue
        vd = (ux, uy, uz)[d] / gamma
        xn = x + vd * dt
        if g.bc[d] == PERIODIC:
            L = g.n[d] * g.dx[d]
            t = xn - g.x0[d]
            t = t - L * np.floor(t / L)
            xn = t + g.x0[d]
        out.append(xn)
    return out


def boris_push(g, pos, u, E, B, qm, dt, valid=None):
    """Relativistic Boris push (the particle push between depositions; the paper's Alg. 1
    leaves it to the host code). Units c = 1, fields at the particles from gather_fields,
    qm the charge-to-mass ratio, h = qm dt / 2:
        u- = u + h E;  t = h B / gamma(u-);  s = 2 t / (1 + |t|^2)
        u' = u- + u- x t;  u+ = u- + u' x s;  u_new = u+ + h E
    u_new is stored as float32; the position then moves with that stored momentum exactly as
    drift() does. Returns (new positions, new momenta as float32 arrays)."""
    pos = _select(pos, valid)
    u = _select(u, valid)
    Ep, Bp = gather_fields(g, pos, E, B)
    h = 0.5 * qm * dt
    um = [np.asarray(u[c], dtype=np.float64) + h * Ep[c] for c in range(3)]
    gm = np.sqrt(1.0 + (um[0] * um[0] + um[1] * um[1]) + um[2] * um[2])
    t = [h * Bp[c] / gm for c in range(3)]
    t2 = (t[0] * t[0] + t[1] * t[1]) + t[2] * t[2]
    sv = [2.0 * t[c] / (1.0 + t2) for c in range(3)]

    def cross(a, b):
        return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]

    c1 = cross(um, t)
    up = [um[c] + c1[c] for c in range(3)]
    c2 = cross(up, sv)
    upl = [um[c] + c2[c] for c in range(3)]
    un = [(upl[c] + h * Ep[c]).astype(np.float32) for c in range(3)]
    return drift(g, [np.asarray(p, dtype=np.float64) for p in pos], un, dt), un


def deposit_midpoint(g, pos, u, w, dt, moved, valid=None):
    """Time-centred current: Eq. 1 evaluated at the midpoint of the step's move x -> x + v dt
    (leapfrog centring; the paper deposits at the stored positions and leaves the push to
    the host code). `moved` says whether `pos` already holds the end of the move (after a
    push: deposit at x - dt v / 2) or its start (the move follows in the same pass: deposit
    at x + dt v / 2). The midpoint is formed with drift() over dt / 2, same operation order
    and periodic wrap."""
    pos = [np.asarray(p, dtype=np.float64) for p in _select(pos[: g.dim], valid)]
    u = _select(u, valid)
    w = _select([w], valid)[0]
    mid = drift(g, pos, u, -0.5 * dt if moved else 0.5 * dt)
    return deposit(g, mid, u, w)
