"""GPU parity of pic_deposit against the FP64 oracle (element-wise over the whole grid)."""
import numpy as np
import pytest
import torch

from gpu_util import TOL_FP32, TOL_SPLIT, oracle_J, rel_l2, say, setup
from paper_2601_08277_amd import synth

pytestmark = pytest.mark.gpu

FP32_PATHS = ["unsorted", "atomic", "cell_valu"]
SPLIT_PATHS = ["mfma_bf16", "mfma_fp16"]


def _cases():
    out = []
    for order in (1, 2, 3):
        out.append((f"periodic-20x18x16-o{order}",
                    lambda o=order: synth.uniform(3, (20, 18, 16), 4, 0.3, o, seed=40 + o)))
        out.append((f"guard-13x11x9-o{order}",
                    lambda o=order: synth.uniform(3, (13, 11, 9), 5, 0.3, o, seed=50 + o,
                                                  bc=(1, 1, 1), ng=3)))
        out.append((f"2d-30x22-o{order}",
                    lambda o=order: synth.uniform(2, (30, 22), 6, 0.2, o, seed=60 + o)))
    out.append(("c1-2d-64x64-o1", synth.c1))
    out.append(("c2-scaled-32^3-o3", lambda: synth.c2(n=(32, 32, 32))))
    return out


CASES = _cases()


def _run(name, make, path, tile=(8, 8, 8)):
    say(f"case {name} path {path}")
    from paper_2601_08277_amd import pic
    params, arrays = make()
    grid, og, parts, bins = setup(params, arrays, tile=tile)
    J = pic.deposit(grid, parts, None if path == "unsorted" else bins, path)
    torch.cuda.synchronize()
    if path != "unsorted":
        bins.check()
    want = oracle_J(og, arrays)
    errs = [rel_l2(J[c].cpu().numpy(), want[c]) for c in range(3)]
    bins.close()
    return errs


@pytest.mark.parametrize("path", FP32_PATHS)
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fp32_paths(case, path):
    errs = _run(case[0], case[1], path)
    assert max(errs) <= TOL_FP32, errs


@pytest.mark.parametrize("path", SPLIT_PATHS)
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_split_paths(case, path):
    errs = _run(case[0], case[1], path)
    assert max(errs) <= TOL_SPLIT, errs


@pytest.mark.parametrize("tile", [(4, 4, 4), (8, 4, 16), (16, 16, 4), (5, 7, 4)])
def test_tile_shapes(tile):
    make = lambda: synth.uniform(3, (21, 17, 12), 6, 0.3, 3, seed=77)
    for path in ("atomic", "cell_valu", "mfma_bf16"):
        errs = _run(f"tile{tile}", make, path, tile=tile)
        tol = TOL_SPLIT if path.startswith("mfma") else TOL_FP32
        assert max(errs) <= tol, (path, errs)


def test_lwfa_shaped_mixed_boundaries():
    """Scaled laser-wakefield snapshot: periodic x, y; guard z; bubble, sheath, ramp."""
    say("case lwfa-32x32x128")
    from paper_2601_08277_amd import pic
    rng = np.random.default_rng(5)
    n = (32, 32, 128)
    counts, sheath = synth.lwfa_counts(n, rng, base_ppc=2.0)
    params, arrays = synth.uniform(3, n, 1, 0.01, 3, seed=6)   # template, replaced below
    x, y, z = synth._place(rng, 3, n, counts)
    N = x.size
    u = [rng.normal(0, 0.05, N), rng.normal(0, 0.05, N), rng.normal(1.0, 0.5, N)]
    arrays = synth._finish(rng, x, y, z, u)
    params = synth._params(3, n, 3, -1.0, (0, 0, 1), 3, 0.2)
    grid, og, parts, bins = setup(params, arrays)
    want = oracle_J(og, arrays)
    for path in ("atomic", "cell_valu", "mfma_bf16", "mfma_fp16"):
        J = pic.deposit(grid, parts, bins, path)
        torch.cuda.synchronize()
        errs = [rel_l2(J[c].cpu().numpy(), want[c]) for c in range(3)]
        tol = TOL_SPLIT if path.startswith("mfma") else TOL_FP32
        assert max(errs) <= tol, (path, errs)
    bins.check()
    bins.close()


def test_empty_and_single_particle():
    from paper_2601_08277_amd import pic
    params, arrays = synth.uniform(3, (9, 9, 9), 1, 0.1, 3, seed=1)
    empty = {k: v[:0] for k, v in arrays.items()}
    grid, og, parts, bins = setup(params, empty)
    J = pic.deposit(grid, parts, bins, "atomic")
    torch.cuda.synchronize()
    assert all(float(j.abs().max()) == 0.0 for j in J)
    bins.close()
    one = {k: v[:1].copy() for k, v in arrays.items()}
    one["x"][:] = 9.0           # exactly on the upper periodic face: clamped cell 8
    one["y"][:] = 0.0
    one["z"][:] = 4.5
    grid, og, parts, bins = setup(params, one)
    want = oracle_J(og, one)
    for path in ("unsorted", "atomic", "cell_valu", "mfma_bf16"):
        J = pic.deposit(grid, parts, None if path == "unsorted" else bins, path)
        torch.cuda.synchronize()
        tol = TOL_SPLIT if path.startswith("mfma") else TOL_FP32
        assert max(rel_l2(J[c].cpu().numpy(), want[c]) for c in range(3)) <= tol, path
    bins.close()


def test_accumulate_flag():
    from paper_2601_08277_amd import pic
    params, arrays = synth.uniform(3, (12, 12, 12), 3, 0.2, 2, seed=3)
    grid, og, parts, bins = setup(params, arrays)
    J = pic.deposit(grid, parts, bins, "atomic")
    J = pic.deposit(grid, parts, bins, "atomic", flags=pic.F_ACCUMULATE, J=J)
    torch.cuda.synchronize()
    want = oracle_J(og, arrays)
    for c in range(3):
        assert rel_l2(J[c].cpu().numpy(), 2 * want[c]) <= TOL_FP32
    bins.close()


def test_out_of_domain_and_nan_are_reported():
    from paper_2601_08277_amd import pic
    params, arrays = synth.uniform(3, (10, 10, 10), 2, 0.1, 1, seed=2, bc=(1, 1, 1), ng=2)
    grid, og, parts, bins = setup(params, arrays)
    parts.x[3] = 10.5            # outside a guard-bounded domain
    J = pic.deposit(grid, parts, bins, "atomic")
    with pytest.raises(pic.PicError) as e:
        bins.check()
    assert e.value.status == -3
    parts.x[3] = float("nan")
    J = pic.deposit(grid, parts, bins, "atomic")
    with pytest.raises(pic.PicError) as e:
        bins.check()
    assert e.value.status == -5
    bins.close()


def test_dense_cells_multiple_units_and_map_windows():
    """A few cells with ~150 particles: a group spans several stage units and several
    slot-map windows; every path still matches the oracle."""
    from paper_2601_08277_amd import pic
    say("case dense cells")
    rng = np.random.default_rng(17)
    n = (12, 12, 12)
    counts = rng.poisson(3.0, size=int(np.prod(n)))
    counts[rng.choice(counts.size, 12, replace=False)] = 150
    x, y, z = synth._place(rng, 3, n, counts)
    u = [rng.normal(0, 0.2, x.size) for _ in range(3)]
    arrays = synth._finish(rng, x, y, z, u)
    params = synth._params(3, n, 3, -1.0, (0, 0, 0), 0, 0.2)
    grid, og, parts, bins = setup(params, arrays, tile=(8, 8, 4))
    want = oracle_J(og, arrays)
    for path in ("cell_valu", "atomic", "mfma_fp16"):
        J = pic.deposit(grid, parts, bins, path)
        torch.cuda.synchronize()
        tol = TOL_SPLIT if path.startswith("mfma") else TOL_FP32
        errs = [rel_l2(J[c].cpu().numpy(), want[c]) for c in range(3)]
        assert max(errs) <= tol, (path, errs)
    rho = pic.deposit_rho(grid, parts, bins)
    torch.cuda.synchronize()
    from oracle import deposit as od
    wr = od.deposit_rho(og, [arrays["x"], arrays["y"], arrays["z"]], arrays["w"])
    assert rel_l2(rho.cpu().numpy(), wr) <= TOL_FP32
    bins.check()
    bins.close()


def test_cell_paths_bitwise_repeatable():
    """The per-cell and split-matrix paths sum in a fixed order (units, flushes, stale list,
    window sum), so two calls on the same bins give the same bits. Checked on freshly sorted
    bins, and with stale particles on a periodic grid that is one tile (every stale
    particle's stencil then lies inside the window; particles that crossed into another tile
    reach J through float atomics, the documented exception)."""
    from paper_2601_08277_amd import pic
    cases = [("32^3 sorted", synth.c2(n=(32, 32, 32)), (8, 8, 4), False),
             ("one tile 8x8x4, stale", synth.uniform(3, (8, 8, 4), 8, 0.3, 3, seed=71),
              (8, 8, 4), True)]
    for name, (params, arrays), tile, stale in cases:
        say(f"case repeatability {name}")
        grid, og, parts, bins = setup(params, arrays, tile=tile, slack=1.0)
        if stale:
            pic.drift(grid, parts, 1.0)
        for path in ("cell_valu", "mfma_bf16"):
            a = pic.deposit(grid, parts, bins, path)
            b = pic.deposit(grid, parts, bins, path)
            torch.cuda.synchronize()
            for c in range(3):
                assert torch.equal(a[c], b[c]), (name, path, c)
        ra = pic.deposit_rho(grid, parts, bins)
        rb = pic.deposit_rho(grid, parts, bins)
        torch.cuda.synchronize()
        assert torch.equal(ra, rb), name
        if stale:
            host = parts.to_numpy()
            valid = host["id"] != -1
            want = oracle_J(og, {k: v[valid] for k, v in host.items()})
            errs = [rel_l2(a[c].cpu().numpy(), want[c]) for c in range(3)]
            assert max(errs) <= TOL_SPLIT, errs
        bins.check()
        bins.close()


def test_unit_cap_boundaries():
    """Units at the 512-particle stage capacity: single cells with 511, 512 and 513
    particles (one unit of a whole cell, then a second unit of one), a 64-cell group with
    exactly 8 per cell (512, one unit) and one with 9 per cell (cut at 8, then 1), and
    empty groups between them; per-cell and split-matrix paths and the charge density
    against the oracle."""
    from paper_2601_08277_amd import pic
    from oracle import deposit as od
    say("case unit cap boundaries")
    rng = np.random.default_rng(23)
    n = (8, 8, 16)                       # four tiles of 8 x 8 x 4, z-planes of 64 cells
    counts = np.zeros(n[::-1], dtype=np.int64)
    counts[1, 2, 3], counts[1, 5, 6], counts[1, 7, 0] = 511, 512, 513   # plane 1
    counts[4, :, :] = 8                  # plane 4: 512 in the group
    counts[9, :, :] = 9                  # plane 9: 576, cut across the cells
    counts[14, :, :] = rng.poisson(8.0, size=(8, 8))
    counts = counts.reshape(-1)
    x, y, z = synth._place(rng, 3, n, counts)
    u = [rng.normal(0, 0.2, x.size) for _ in range(3)]
    arrays = synth._finish(rng, x, y, z, u)
    params = synth._params(3, n, 3, -1.0, (0, 0, 0), 0, 0.2)
    grid, og, parts, bins = setup(params, arrays, tile=(8, 8, 4), slack=0.5)
    want = oracle_J(og, arrays)
    for path in ("cell_valu", "mfma_fp16"):
        J = pic.deposit(grid, parts, bins, path)
        torch.cuda.synchronize()
        tol = TOL_SPLIT if path.startswith("mfma") else TOL_FP32
        errs = [rel_l2(J[c].cpu().numpy(), want[c]) for c in range(3)]
        assert max(errs) <= tol, (path, errs)
    rho = pic.deposit_rho(grid, parts, bins)
    torch.cuda.synchronize()
    wr = od.deposit_rho(og, [arrays["x"], arrays["y"], arrays["z"]], arrays["w"])
    assert rel_l2(rho.cpu().numpy(), wr) <= TOL_FP32
    bins.check()
    bins.close()
