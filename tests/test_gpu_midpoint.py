"""GPU parity of the time-centred current (PIC_F_MIDPOINT) against the FP64 oracle.

Deposition at the midpoint of the move: from the end of a move already made (x - v dt/2),
or from its start with the move done in the same pass (PIC_F_DRIFT, x + v dt/2). Particles
whose midpoint cell differs from their bin take the stale path, which these inputs
exercise (|u| ~ 0.3, dt up to 1)."""
import numpy as np
import pytest
import torch

from gpu_util import TOL_FP32, check_bins, rel_l2, say, setup
from oracle import deposit as od
from paper_2601_08277_amd import synth

pytestmark = pytest.mark.gpu


CASES = []
for _o in (1, 2, 3):
    CASES.append((f"periodic-20x18x16-o{_o}",
                  lambda o=_o: synth.uniform(3, (20, 18, 16), 4, 0.3, o, seed=440 + o, dt=0.9)))
    CASES.append((f"2d-30x22-o{_o}",
                  lambda o=_o: synth.uniform(2, (30, 22), 6, 0.3, o, seed=460 + o, dt=0.7)))
CASES.append(("c2-scaled-32^3-o3", lambda: synth.c2(n=(32, 32, 32))))


def _oracle(og, arrays, dt, moved):
    pos = [arrays["x"], arrays["y"], arrays["z"]]
    u = [arrays["ux"], arrays["uy"], arrays["uz"]]
    return od.deposit_midpoint(og, pos, u, arrays["w"], dt, moved)


@pytest.mark.parametrize("drift", [False, True], ids=["after-push", "fused-drift"])
@pytest.mark.parametrize("path", ["cell_valu", "unsorted"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_midpoint_matches_oracle(case, path, drift):
    from paper_2601_08277_amd import pic
    say(f"case midpoint {case[0]} {path} drift={drift}")
    params, arrays = case[1]()
    grid, og, parts, bins = setup(params, arrays, tile=(8, 8, 4))
    fl = pic.F_MIDPOINT | (pic.F_DRIFT if drift else 0)
    J = pic.deposit(grid, parts, None if path == "unsorted" else bins, path, fl)
    torch.cuda.synchronize()
    bins.check()
    want = _oracle(og, arrays, params["dt"], moved=not drift)
    errs = [rel_l2(J[c].cpu().numpy(), want[c]) for c in range(3)]
    assert max(errs) <= TOL_FP32, errs
    host = parts.to_numpy()
    valid = host["id"] != -1
    order = np.argsort(host["id"][valid])
    pos = [arrays["x"], arrays["y"], arrays["z"]]
    u = [arrays["ux"], arrays["uy"], arrays["uz"]]
    end = od.drift(og, pos, u, params["dt"]) if drift else pos
    for d, name in enumerate(("x", "y", "z")[: og.dim]):
        assert np.array_equal(host[name][valid][order], end[d]), name
    bins.close()


def test_midpoint_fused_drift_movers_then_rebin():
    """DRIFT | EMIT_MOVERS | MIDPOINT: movers are found against the moved positions and
    the incremental rebin that consumes them leaves valid bins."""
    from paper_2601_08277_amd import pic
    say("case midpoint movers + rebin")
    params, arrays = synth.uniform(3, (24, 16, 16), 6, 0.3, 3, seed=470, dt=0.8)
    grid, og, parts, bins = setup(params, arrays, tile=(8, 8, 4), slack=0.5)
    pos = [arrays["x"], arrays["y"], arrays["z"]]
    u = [arrays["ux"], arrays["uy"], arrays["uz"]]
    for step in range(3):
        J = pic.deposit(grid, parts, bins, "cell_valu",
                        pic.F_DRIFT | pic.F_EMIT_MOVERS | pic.F_MIDPOINT)
        torch.cuda.synchronize()
        bins.check()
        want = od.deposit_midpoint(og, pos, u, arrays["w"], params["dt"], moved=False)
        errs = [rel_l2(J[c].cpu().numpy(), want[c]) for c in range(3)]
        assert max(errs) <= TOL_FP32, (step, errs)
        pos = od.drift(og, pos, u, params["dt"])
        pic.rebin(grid, parts, bins, pic.REBIN_INCREMENTAL)
        st = bins.stats()
        assert st["n_moved"] > 0
        off, ln, bc = bins.tables()
        check_bins(og, parts.to_numpy(), off, ln, bc,
                   stale_ok=st["n_overflow"] + st["n_mover_drop"])
    bins.close()


def test_midpoint_batched_matches_single_patch():
    from paper_2601_08277_amd import pic
    patches = synth.c4_patches(npatch=4, edge=(8, 20), ppc_clip=(1, 24), seed=17)
    for params, _ in patches:
        params["dt"] = 0.6
        params["bc"] = (0, 0, 0)
        params["ng"] = 0
    say("case midpoint batched")
    a = [setup(p, ar, tile=(4, 4, 4)) for p, ar in patches]
    b = [setup(p, ar, tile=(4, 4, 4)) for p, ar in patches]
    plan = pic.Plan([m[0] for m in a], [m[3] for m in a])
    fl = pic.F_MIDPOINT | pic.F_DRIFT
    Jb = pic.deposit_batched(plan, [m[2] for m in a], flags=fl)
    Js = [pic.deposit(m[0], m[2], m[3], "cell_valu", fl) for m in b]
    torch.cuda.synchronize()
    for k, (params, arrays) in enumerate(patches):
        # particles whose midpoint leaves their tile's window are added with global atomics,
        # whose order differs between launches: equal to float32 rounding, not bitwise
        for c in range(3):
            assert rel_l2(Jb[k][c].cpu().numpy(), Js[k][c].cpu().numpy()) <= TOL_FP32
        for name in ("x", "y", "z"):
            assert torch.equal(getattr(a[k][2], name), getattr(b[k][2], name))
        want = _oracle(a[k][1], arrays, 0.6, moved=False)
        errs = [rel_l2(Jb[k][c].cpu().numpy(), want[c]) for c in range(3)]
        assert max(errs) <= TOL_FP32, (k, errs)
    plan.close()
    for m in a + b:
        m[3].close()


def test_midpoint_refused_on_other_paths():
    from paper_2601_08277_amd import pic
    say("case midpoint refused")
    params, arrays = synth.uniform(3, (8, 8, 8), 2, 0.3, 1, seed=480, dt=0.5)
    grid, og, parts, bins = setup(params, arrays, tile=(4, 4, 4))
    for path in ("atomic", "mfma_bf16"):
        with pytest.raises(pic.PicError) as e:
            pic.deposit(grid, parts, bins, path, pic.F_MIDPOINT)
        assert e.value.status == pic.PIC_ERR_UNSUPPORTED
    bins.close()
