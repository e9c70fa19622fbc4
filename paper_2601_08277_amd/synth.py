"""Seeded synthetic particle workloads (no deposition arithmetic lives here).

These stand in for the WarpX input decks of the paper (uniform plasma and laser
wakefield, Appendix A), which are not available. Every generator returns

    params: dict(dim, n, order, q, bc, ng, dt, x0, dx)
    arrays: dict(x, y, z: float64; ux, uy, uz, w: float32; id: int32)

Positions are cell index + U[0, 1) per dimension in float64, generated in cell order
and then shuffled with the same generator, so a first global sort is a real sort.
Momenta are drawn in float64 and rounded to float32 storage; consumers promote the
stored float32 values. Generator: numpy.random.default_rng(seed).

The same module feeds the library and the CPU oracle; it computes nothing the method
computes (no cells, weights, velocities or drifts).
"""
import numpy as np

PERIODIC = 0
GUARD = 1


def _params(dim, n, order, q=-1.0, bc=(PERIODIC,) * 3, ng=0, dt=0.0):
    n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
    return dict(dim=int(dim), n=n, order=int(order), q=float(q), bc=tuple(bc), ng=int(ng),
                dt=float(dt), x0=(0.0, 0.0, 0.0), dx=(1.0, 1.0, 1.0))


def _place(rng, dim, n, counts):
    """Positions for `counts[c]` particles in each cell c (x-fastest), in cell order."""
    counts = np.asarray(counts, dtype=np.int64).reshape(-1)
    cells = np.repeat(np.arange(counts.size, dtype=np.int64), counts)
    nx, ny = n[0], n[1]
    i = cells % nx
    j = (cells // nx) % ny
    k = cells // (nx * ny)
    N = cells.size
    x = i.astype(np.float64) + rng.random(N)
    y = j.astype(np.float64) + rng.random(N)
    z = k.astype(np.float64) + rng.random(N) if dim == 3 else np.zeros(N)
    return x, y, z


def _finish(rng, x, y, z, u, w=1.0):
    """Shuffle, round momenta to float32, assign ids 0..N-1 (id = index after shuffle)."""
    N = x.size
    perm = rng.permutation(N)
    arrays = dict(x=np.ascontiguousarray(x[perm]), y=np.ascontiguousarray(y[perm]),
                  z=np.ascontiguousarray(z[perm]),
                  ux=u[0][perm].astype(np.float32), uy=u[1][perm].astype(np.float32),
                  uz=u[2][perm].astype(np.float32),
                  w=np.full(N, w, dtype=np.float32),
                  id=np.arange(N, dtype=np.int32))
    return arrays


def uniform(dim, n, ppc, u_sigma, order, seed, q=-1.0, bc=None, ng=0, dt=0.0):
    """Uniform plasma: exactly `ppc` particles per cell, u ~ N(0, u_sigma) per component."""
    rng = np.random.default_rng(seed)
    n3 = tuple(n) + (1,) * (3 - len(n))
    ncell = int(np.prod(n3[:dim]))
    x, y, z = _place(rng, dim, n3, np.full(ncell, ppc))
    N = x.size
    u = [rng.normal(0.0, u_sigma, N) for _ in range(3)]
    bc = bc if bc is not None else (PERIODIC,) * 3
    return _params(dim, n3, order, q, bc, ng, dt), _finish(rng, x, y, z, u)


def c1():
    """2D3V, 64 x 64 periodic, 16 particles per cell, u ~ N(0, 0.01), order 1, dt 0.5."""
    return uniform(2, (64, 64), 16, 0.01, 1, seed=1001, dt=0.5)


def c2(n=(128, 128, 128), ppc=8):
    """3D3V uniform plasma, 128^3 periodic, 8 per cell, u ~ N(0, 0.05), order 3, dt 0.2."""
    return uniform(3, n, ppc, 0.05, 3, seed=1002, dt=0.2)


def lwfa_counts(n, rng, base_ppc=2.0):
    """Per-cell particle counts of the laser-wakefield-shaped snapshot.

    Density n(r) = ramp(z) * m(r) at cell centres: ramp rises linearly from 0 to 1 over
    the first 10 % of z; m = 0 inside an ellipsoidal bubble centred at
    (nx/2, ny/2, 3 nz/4) with semi-axes (3 nx/16, 3 ny/16, 3 nz/32), m = 5 in a shell
    6 cells thick around it (the sheath), m = 1 elsewhere (drive region and background).
    Count = stochastic rounding of base_ppc * n. Returns (counts, sheath mask), x fastest.
    """
    nx, ny, nz = n
    cz, cy, cx = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                             indexing="ij")
    ramp = np.minimum(1.0, cz / (0.1 * nz))
    ax, ay, az = 3.0 * nx / 16.0, 3.0 * ny / 16.0, 3.0 * nz / 32.0
    ox, oy, oz = nx / 2.0, ny / 2.0, 3.0 * nz / 4.0
    r_in = ((cx - ox) / ax) ** 2 + ((cy - oy) / ay) ** 2 + ((cz - oz) / az) ** 2
    r_out = ((cx - ox) / (ax + 6)) ** 2 + ((cy - oy) / (ay + 6)) ** 2 + ((cz - oz) / (az + 6)) ** 2
    m = np.where(r_in < 1.0, 0.0, np.where(r_out < 1.0, 5.0, 1.0))
    dens = base_ppc * ramp * m
    fl = np.floor(dens)
    counts = (fl + (rng.random(dens.shape) < (dens - fl))).astype(np.int64)
    sheath = (r_in >= 1.0) & (r_out < 1.0)
    return counts.reshape(-1), sheath.reshape(-1)


def c3(n=(256, 256, 1024), ng=3):
    """3D laser-wakefield-shaped snapshot, order 3, periodic in x and y, guard in z.

    Background u ~ N(0, 0.01); in the sheath u_z ~ N(2, 0.5) and u_x, u_y ~ N(0, 0.05).
    """
    rng = np.random.default_rng(1003)
    counts, sheath = lwfa_counts(n, rng)
    x, y, z = _place(rng, 3, n, counts)
    N = x.size
    in_sheath = np.repeat(sheath, counts)
    ux = np.where(in_sheath, rng.normal(0.0, 0.05, N), rng.normal(0.0, 0.01, N))
    uy = np.where(in_sheath, rng.normal(0.0, 0.05, N), rng.normal(0.0, 0.01, N))
    uz = np.where(in_sheath, rng.normal(2.0, 0.5, N), rng.normal(0.0, 0.01, N))
    params = _params(3, n, 3, -1.0, (PERIODIC, PERIODIC, GUARD), ng, 0.2)
    return params, _finish(rng, x, y, z, [ux, uy, uz])


def c4_patches(npatch=64, edge=(32, 96), ppc_mu=np.log(8.0), ppc_sigma=1.0,
               ppc_clip=(1, 64), ng=3, u_sigma=0.05, seed=1004):
    """Batched uneven patches: independent 3D guard-bounded patches.

    Edge lengths uniform in {edge[0]..edge[1]} per dimension, particles per cell
    clip(rint(lognormal(ppc_mu, ppc_sigma)), ppc_clip), order uniform in {1, 2, 3}.
    Returns a list of (params, arrays).
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(npatch):
        n = tuple(int(v) for v in rng.integers(edge[0], edge[1] + 1, size=3))
        ppc = int(np.clip(np.rint(rng.lognormal(ppc_mu, ppc_sigma)), *ppc_clip))
        order = int(rng.integers(1, 4))
        prng = np.random.default_rng(rng.integers(0, 2 ** 63 - 1))
        x, y, z = _place(prng, 3, n, np.full(int(np.prod(n)), ppc))
        N = x.size
        u = [prng.normal(0.0, u_sigma, N) for _ in range(3)]
        params = _params(3, n, order, -1.0, (GUARD,) * 3, ng, 0.0)
        params["ppc"] = ppc
        out.append((params, _finish(prng, x, y, z, u)))
    return out


def c5(n=(64, 64, 64), ppc=8):
    """Adjoint check: 64^3 periodic, 8 per cell, order 3, u ~ N(0, 0.05)."""
    return uniform(3, n, ppc, 0.05, 3, seed=1005)


def adjoint_field(shape, seed=1005):
    """dL/dJ for L = sum J . G: three float32 grids with entries ~ N(0, 1)."""
    rng = np.random.default_rng(seed + 10_000)
    return [rng.normal(0.0, 1.0, shape).astype(np.float32) for _ in range(3)]


def sample_indices(N, k, seed):
    """k distinct particle indices, drawn without replacement."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(N, size=min(k, N), replace=False))
