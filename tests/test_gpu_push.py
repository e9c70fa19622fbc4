"""GPU parity of pic_push (gather + Boris rotation + move) against the FP64 oracle.

Error budget: the fields are gathered in float32 (relative error ~1e-6 of the gathered
value), the rotation runs in float64 and u is rounded to float32, so |du| stays below
h (|dE| + |u| |dB|) + ulp(u) with h = qm dt / 2; positions move by dt times that."""
import numpy as np
import pytest
import torch

from gpu_util import say, setup
from oracle import deposit as od
from paper_2601_08277_amd import synth

pytestmark = pytest.mark.gpu

QM, DT = -1.0, 0.3


def _fields(shape, seed, e_sigma=0.1, b_sigma=1.0):
    rng = np.random.default_rng(seed)
    E = [rng.normal(0, e_sigma, shape).astype(np.float32) for _ in range(3)]
    B = [rng.normal(0, b_sigma, shape).astype(np.float32) for _ in range(3)]
    return E, B


def _check_against_oracle(og, before, after, valid, E, B, qm, dt, tol_u=5e-6, tol_x=1e-5):
    pos = [before["x"], before["y"], before["z"]]
    u = [before["ux"], before["uy"], before["uz"]]
    wpos, wu = od.boris_push(og, pos, u, [e.astype(np.float64) for e in E],
                             [b.astype(np.float64) for b in B], qm, dt, valid=valid)
    for c, name in enumerate(("ux", "uy", "uz")):
        got = after[name][valid].astype(np.float64)
        want = wu[c].astype(np.float64)
        err = np.abs(got - want)
        bound = tol_u * (1.0 + np.abs(want))
        assert np.all(err <= bound), f"{name}: max excess {np.max(err - bound)}"
    for d, name in enumerate(("x", "y", "z")[: og.dim]):
        diff = after[name][valid] - wpos[d]
        if og.bc[d] == od.PERIODIC:
            L = og.n[d] * og.dx[d]
            diff = diff - L * np.round(diff / L)
        assert np.max(np.abs(diff)) <= tol_x * og.dx[d], f"{name}: {np.max(np.abs(diff))}"
    for name in ("x", "y", "z", "ux", "uy", "uz"):
        assert np.array_equal(after[name][~valid], before[name][~valid]), f"gap slot {name} changed"


CASES = []
for _o in (1, 2, 3):
    CASES.append((f"periodic-18x16x14-o{_o}",
                  lambda o=_o: synth.uniform(3, (18, 16, 14), 3, 0.3, o, seed=340 + o)))
    CASES.append((f"guard-13x11x9-o{_o}",
                  lambda o=_o: synth.uniform(3, (13, 11, 9), 4, 0.3, o, seed=350 + o,
                                             bc=(1, 1, 1), ng=3)))
    CASES.append((f"2d-30x22-o{_o}",
                  lambda o=_o: synth.uniform(2, (30, 22), 5, 0.2, o, seed=360 + o)))


@pytest.mark.parametrize("with_bins", [True, False])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_push_matches_oracle(case, with_bins):
    from paper_2601_08277_amd import pic
    say(f"case push {case[0]} bins={with_bins}")
    params, arrays = case[1]()
    grid, og, parts, bins = setup(params, arrays, tile=(8, 8, 4))
    E, B = _fields(grid.shape, 11)
    before = parts.to_numpy()
    pic.push(grid, parts, bins if with_bins else None,
             [torch.from_numpy(e).cuda() for e in E], [torch.from_numpy(b).cuda() for b in B],
             QM, DT)
    torch.cuda.synchronize()
    bins.check()
    after = parts.to_numpy()
    _check_against_oracle(og, before, after, before["id"] != -1, E, B, QM, DT)
    bins.close()


def test_push_with_stale_bins():
    """Particles moved away from their tiles without a rebin take the global path."""
    from paper_2601_08277_amd import pic
    say("case push stale")
    params, arrays = synth.uniform(3, (16, 12, 12), 4, 0.4, 3, seed=43)
    grid, og, parts, bins = setup(params, arrays, tile=(4, 4, 4))
    pic.drift(grid, parts, 2.5)
    E, B = _fields(grid.shape, 12)
    before = parts.to_numpy()
    pic.push(grid, parts, bins, [torch.from_numpy(e).cuda() for e in E],
             [torch.from_numpy(b).cuda() for b in B], QM, DT)
    torch.cuda.synchronize()
    bins.check()
    _check_against_oracle(og, before, parts.to_numpy(), before["id"] != -1, E, B, QM, DT)
    bins.close()


def test_push_then_rebin_steps():
    """Five push + incremental rebin steps; each step checked from the GPU's own state."""
    from paper_2601_08277_amd import pic
    say("case push steps")
    params, arrays = synth.uniform(3, (20, 16, 12), 6, 0.3, 2, seed=44)
    grid, og, parts, bins = setup(params, arrays, tile=(8, 8, 4), slack=0.5)
    E, B = _fields(grid.shape, 13)
    Et = [torch.from_numpy(e).cuda() for e in E]
    Bt = [torch.from_numpy(b).cuda() for b in B]
    n0 = int(np.count_nonzero(parts.to_numpy()["id"] != -1))
    for step in range(5):
        before = parts.to_numpy()
        pic.push(grid, parts, bins, Et, Bt, QM, 0.8)
        torch.cuda.synchronize()
        _check_against_oracle(og, before, parts.to_numpy(), before["id"] != -1, E, B, QM, 0.8)
        pic.rebin(grid, parts, bins, pic.REBIN_INCREMENTAL)
        bins.check()
        assert int(np.count_nonzero(parts.to_numpy()["id"] != -1)) == n0
    bins.close()


def test_push_uniform_b_keeps_speed():
    """A uniform B with E = 0 rotates u about B: |u| is kept to float32 rounding."""
    from paper_2601_08277_amd import pic
    say("case push uniform B")
    params, arrays = synth.uniform(3, (32, 32, 32), 8, 0.3, 3, seed=45)
    grid, og, parts, bins = setup(params, arrays, tile=(8, 8, 4))
    shape = grid.shape
    Et = [torch.zeros(shape, device="cuda") for _ in range(3)]
    Bt = [torch.full(shape, v, device="cuda") for v in (0.3, -0.6, 0.9)]
    before = parts.to_numpy()
    for _ in range(10):
        pic.push(grid, parts, bins, Et, Bt, QM, DT)
    torch.cuda.synchronize()
    after = parts.to_numpy()
    valid = before["id"] != -1
    sp = lambda h: np.sqrt(sum(h[n][valid].astype(np.float64) ** 2 for n in ("ux", "uy", "uz")))
    np.testing.assert_allclose(sp(after), sp(before), rtol=2e-6, atol=1e-7)
    bpar = lambda h: (0.3 * h["ux"][valid] - 0.6 * h["uy"][valid] + 0.9 * h["uz"][valid])
    np.testing.assert_allclose(bpar(after), bpar(before), rtol=0, atol=2e-6)
    bins.close()


def test_push_full_size_sampled():
    """128^3 cells, 8 per cell, order 3 (the uniform-plasma workload): every particle
    pushed on the GPU, a sample of 4096 checked against the oracle."""
    from paper_2601_08277_amd import pic
    say("case push full size")
    params, arrays = synth.c2()
    grid, og, parts, bins = setup(params, arrays, tile=(8, 8, 4), slack=0.5)
    E, B = _fields(grid.shape, 14)
    before = parts.to_numpy()
    pic.push(grid, parts, bins, [torch.from_numpy(e).cuda() for e in E],
             [torch.from_numpy(b).cuda() for b in B], QM, params["dt"])
    torch.cuda.synchronize()
    bins.check()
    after = parts.to_numpy()
    valid_slots = np.flatnonzero(before["id"] != -1)
    rng = np.random.default_rng(5)
    pick = np.zeros(before["id"].size, bool)
    pick[rng.choice(valid_slots, 4096, replace=False)] = True
    sub = lambda h: {k: v[pick] for k, v in h.items()}
    sb, sa = sub(before), sub(after)
    _check_against_oracle(og, sb, sa, np.ones(4096, bool), E, B, QM, params["dt"])
    bins.close()
