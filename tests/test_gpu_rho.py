"""GPU parity of pic_deposit_rho against the FP64 charge-density oracle."""
import numpy as np
import pytest
import torch

from gpu_util import TOL_FP32, rel_l2, say, setup
from oracle import deposit as od
from paper_2601_08277_amd import synth

pytestmark = pytest.mark.gpu


def _cases():
    out = []
    for order in (1, 2, 3):
        out.append((f"periodic-20x18x16-o{order}",
                    lambda o=order: synth.uniform(3, (20, 18, 16), 4, 0.3, o, seed=140 + o)))
        out.append((f"guard-13x11x9-o{order}",
                    lambda o=order: synth.uniform(3, (13, 11, 9), 5, 0.3, o, seed=150 + o,
                                                  bc=(1, 1, 1), ng=3)))
        out.append((f"2d-30x22-o{order}",
                    lambda o=order: synth.uniform(2, (30, 22), 6, 0.2, o, seed=160 + o)))
    out.append(("c2-scaled-32^3-o3", lambda: synth.c2(n=(32, 32, 32))))
    return out


CASES = _cases()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_rho_matches_oracle(case):
    from paper_2601_08277_amd import pic
    say(f"case rho {case[0]}")
    params, arrays = case[1]()
    grid, og, parts, bins = setup(params, arrays, tile=(8, 8, 4))
    rho = pic.deposit_rho(grid, parts, bins)
    torch.cuda.synchronize()
    bins.check()
    want = od.deposit_rho(og, [arrays["x"], arrays["y"], arrays["z"]], arrays["w"])
    assert rel_l2(rho.cpu().numpy(), want) <= TOL_FP32
    rho2 = pic.deposit_rho(grid, parts, bins, flags=pic.F_ACCUMULATE, rho=rho)
    torch.cuda.synchronize()
    assert rel_l2(rho2.cpu().numpy(), 2 * want) <= TOL_FP32
    bins.close()


def test_rho_with_stale_bins():
    """Movers left in full bins (slack 0) go through the stale end phase."""
    from paper_2601_08277_amd import pic
    say("case rho stale")
    params, arrays = synth.uniform(3, (16, 12, 12), 4, 0.4, 3, seed=31)
    grid, og, parts, bins = setup(params, arrays, tile=(4, 4, 4), slack=0.0)
    pic.drift(grid, parts, 1.5)
    pic.rebin(grid, parts, bins, pic.REBIN_INCREMENTAL)
    assert bins.stats()["n_overflow"] > 0
    rho = pic.deposit_rho(grid, parts, bins)
    torch.cuda.synchronize()
    host = parts.to_numpy()
    valid = host["id"] != -1
    want = od.deposit_rho(og, [host["x"], host["y"], host["z"]], host["w"], valid=valid)
    assert rel_l2(rho.cpu().numpy(), want) <= TOL_FP32
    bins.check()
    bins.close()


def test_rho_rejects_drift_flags():
    from paper_2601_08277_amd import pic
    params, arrays = synth.uniform(3, (8, 8, 8), 2, 0.1, 1, seed=2)
    grid, og, parts, bins = setup(params, arrays, tile=(4, 4, 4))
    with pytest.raises(pic.PicError) as e:
        pic.deposit_rho(grid, parts, bins, flags=pic.F_DRIFT)
    assert e.value.status == pic.PIC_ERR_INVALID_ARG
    bins.close()
