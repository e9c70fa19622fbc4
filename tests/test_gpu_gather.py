"""GPU parity of pic_gather_fields against the FP64 field-gather oracle."""
import numpy as np
import pytest
import torch

from gpu_util import TOL_FP32, rel_l2, say, setup
from oracle import deposit as od
from paper_2601_08277_amd import synth

pytestmark = pytest.mark.gpu


def _fields(shape, seed):
    rng = np.random.default_rng(seed)
    return [rng.normal(size=shape).astype(np.float32) for _ in range(6)]


CASES = []
for _o in (1, 2, 3):
    CASES.append((f"periodic-18x16x14-o{_o}",
                  lambda o=_o: synth.uniform(3, (18, 16, 14), 3, 0.3, o, seed=240 + o)))
    CASES.append((f"guard-13x11x9-o{_o}",
                  lambda o=_o: synth.uniform(3, (13, 11, 9), 4, 0.3, o, seed=250 + o,
                                             bc=(1, 1, 1), ng=3)))
    CASES.append((f"2d-30x22-o{_o}",
                  lambda o=_o: synth.uniform(2, (30, 22), 5, 0.2, o, seed=260 + o)))


@pytest.mark.parametrize("with_bins", [True, False])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_gather_matches_oracle(case, with_bins):
    from paper_2601_08277_amd import pic
    say(f"case gather {case[0]} bins={with_bins}")
    params, arrays = case[1]()
    grid, og, parts, bins = setup(params, arrays, tile=(8, 8, 4))
    F = _fields(grid.shape, 7)
    Ft = [torch.from_numpy(f).cuda() for f in F]
    Ep, Bp = pic.gather_fields(grid, parts, bins if with_bins else None, Ft[:3], Ft[3:])
    torch.cuda.synchronize()
    bins.check()
    ids = parts.id.cpu().numpy()
    valid = ids != -1
    order = np.argsort(ids[valid])
    wE, wB = od.gather_fields(og, [arrays["x"], arrays["y"], arrays["z"]],
                              [f.astype(np.float64) for f in F[:3]],
                              [f.astype(np.float64) for f in F[3:]])
    for got, want in zip(Ep + Bp, wE + wB):
        g = got.cpu().numpy()
        assert rel_l2(g[valid][order], want) <= TOL_FP32
        assert np.all(g[~valid] == 0)
    bins.close()


def test_gather_with_stale_bins():
    from paper_2601_08277_amd import pic
    say("case gather stale")
    params, arrays = synth.uniform(3, (16, 12, 12), 4, 0.4, 3, seed=41)
    grid, og, parts, bins = setup(params, arrays, tile=(4, 4, 4), slack=0.0)
    pic.drift(grid, parts, 1.5)
    pic.rebin(grid, parts, bins, pic.REBIN_INCREMENTAL)
    assert bins.stats()["n_overflow"] > 0
    F = _fields(grid.shape, 9)
    Ft = [torch.from_numpy(f).cuda() for f in F]
    Ep, Bp = pic.gather_fields(grid, parts, bins, Ft[:3], Ft[3:])
    torch.cuda.synchronize()
    host = parts.to_numpy()
    valid = host["id"] != -1
    wE, wB = od.gather_fields(og, [host["x"], host["y"], host["z"]],
                              [f.astype(np.float64) for f in F[:3]],
                              [f.astype(np.float64) for f in F[3:]], valid=valid)
    for got, want in zip(Ep + Bp, wE + wB):
        assert rel_l2(got.cpu().numpy()[valid], want) <= TOL_FP32
    bins.check()
    bins.close()
