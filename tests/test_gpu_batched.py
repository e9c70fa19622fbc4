"""Batched persistent deposition over uneven patches (pic_deposit_batched).

Each patch's J must equal the single-patch pic_deposit bitwise (same per-tile arithmetic
and window sum) and the FP64 oracle to the float32 tolerance; graph replays must equal the
eager call bitwise.
"""
import numpy as np
import pytest
import torch

from gpu_util import TOL_FP32, check_bins, oracle_J, rel_l2, say, setup
from paper_2601_08277_amd import synth

pytestmark = pytest.mark.gpu


def _patches(npatch=6, seed=7):
    # C4's recipe at small edges: U{8..20} cells, ppc lognormal(ln 8, 1) clipped to [1, 24]
    return synth.c4_patches(npatch=npatch, edge=(8, 20), ppc_clip=(1, 24), seed=seed)


def _make(patches, tile=(4, 4, 4)):
    made = []
    for params, arrays in patches:
        made.append(setup(params, arrays, tile=tile))
    return made


def test_batched_matches_single_patch_and_oracle():
    from paper_2601_08277_amd import pic
    patches = _patches()
    say("case batched 6 patches, mixed orders")
    made = _make(patches)
    plan = pic.Plan([m[0] for m in made], [m[3] for m in made])
    info = plan.info()
    assert info["items"] == sum(m[3].view().ntiles for m in made)
    Jb = pic.deposit_batched(plan, [m[2] for m in made])
    torch.cuda.synchronize()
    for k, ((params, arrays), (grid, og, parts, bins)) in enumerate(zip(patches, made)):
        Js = pic.deposit(grid, parts, bins, "cell_valu")
        torch.cuda.synchronize()
        bins.check()
        for c in range(3):
            assert torch.equal(Jb[k][c], Js[c]), (k, c, params["order"])
        want = oracle_J(og, arrays)
        errs = [rel_l2(Jb[k][c].cpu().numpy(), want[c]) for c in range(3)]
        assert max(errs) <= TOL_FP32, (k, params["order"], errs)
    plan.close()
    for m in made:
        m[3].close()


def test_batched_drift_and_movers_match_single_patch():
    from paper_2601_08277_amd import pic
    patches = _patches(npatch=4, seed=11)
    for params, _ in patches:      # periodic, so the drift cannot leave the patch
        params["dt"] = 0.5
        params["bc"] = (0, 0, 0)
        params["ng"] = 0
    say("case batched drift + movers")
    a = _make(patches)
    b = _make(patches)
    plan = pic.Plan([m[0] for m in a], [m[3] for m in a])
    fl = pic.F_DRIFT | pic.F_EMIT_MOVERS
    Jb = pic.deposit_batched(plan, [m[2] for m in a], flags=fl)
    Js = [pic.deposit(m[0], m[2], m[3], "cell_valu", fl) for m in b]
    torch.cuda.synchronize()
    for k in range(len(patches)):
        for c in range(3):
            assert torch.equal(Jb[k][c], Js[k][c])
        for name in ("x", "y", "z"):
            assert torch.equal(getattr(a[k][2], name), getattr(b[k][2], name))
        # the incremental rebin that consumes the movers gives the same bins
        pic.rebin(a[k][0], a[k][2], a[k][3], pic.REBIN_INCREMENTAL)
        pic.rebin(b[k][0], b[k][2], b[k][3], pic.REBIN_INCREMENTAL)
        sa, sb = a[k][3].stats(), b[k][3].stats()
        assert sa["n_moved"] == sb["n_moved"] > 0
        assert sa["n_valid"] == sb["n_valid"]
        # which inserts find a full bin depends on the (unordered) mover list, so the
        # bins are compared through the sorter invariants, not slot by slot
        for m, st in ((a[k], sa), (b[k], sb)):
            off, ln, bc = m[3].tables()
            host = m[2].to_numpy()
            check_bins(m[1], host, off, ln, bc, stale_ok=st["n_overflow"] + st["n_mover_drop"])
    plan.close()
    for m in a + b:
        m[3].close()


def test_batched_graph_replays_equal_eager():
    from paper_2601_08277_amd import pic
    patches = _patches(npatch=5, seed=13)
    say("case batched graph capture")
    made = _make(patches)
    plan = pic.Plan([m[0] for m in made], [m[3] for m in made])
    parts = [m[2] for m in made]
    J = pic.deposit_batched(plan, parts)              # eager call uploads the descriptors
    torch.cuda.synchronize()
    ref = [[j.clone() for j in Jk] for Jk in J]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pic.deposit_batched(plan, parts, J)
    torch.cuda.synchronize()
    for rep in range(3):
        for Jk in J:                                   # eager work between replays
            for j in Jk:
                j.fill_(float(rep + 1))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in range(len(patches)):
            for c in range(3):
                assert torch.equal(J[k][c], ref[k][c]), (rep, k, c)
    plan.close()
    for m in made:
        m[3].close()


def test_batched_argument_errors():
    from paper_2601_08277_amd import pic
    (p3, a3), = synth.c4_patches(npatch=1, edge=(8, 10), ppc_clip=(1, 4), seed=3)
    g3, _, parts3, bins3 = setup(p3, a3, tile=(4, 4, 4))
    p2, a2 = synth.uniform(2, (16, 16), 2, 0.1, 1, seed=4)
    g2, _, parts2, bins2 = setup(p2, a2, tile=(4, 4))
    with pytest.raises(pic.PicError) as e:
        pic.Plan([g2], [bins2])
    assert e.value.status == pic.PIC_ERR_UNSUPPORTED
    p3b = dict(p3)
    p3b["n"] = (p3["n"][0] + 1,) + tuple(p3["n"][1:])
    with pytest.raises(pic.PicError) as e:
        pic.Plan([pic.Grid(p3b)], [bins3])
    assert e.value.status == pic.PIC_ERR_INVALID_ARG
    plan = pic.Plan([g3], [bins3])
    with pytest.raises(pic.PicError) as e:
        pic.deposit_batched(plan, [parts3], path="mfma_bf16")
    assert e.value.status == pic.PIC_ERR_UNSUPPORTED
    plan.close()
    bins2.close()
    bins3.close()


def test_batched_with_tuned_tiles_and_launch_shape():
    """The C4 recipe at larger edges, each patch binned with the tile the committed tuning
    cache gives its (order, ppc) and the plan built with the cache's workgroups per compute
    unit: every patch matches the oracle and the single-patch call bitwise."""
    import os
    from paper_2601_08277_amd import autotune, pic
    cache_path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                              "paper_2601_08277_amd", "tune_cache.json")
    cache = autotune.load(cache_path)
    patches = synth.c4_patches(npatch=6, edge=(16, 40), ppc_clip=(1, 40), seed=17)
    say("case batched tuned tiles")
    made, tiles = [], []
    for params, arrays in patches:
        tile = autotune.lookup(cache, params["order"], params["ppc"])[0]
        tiles.append(tile)
        made.append(setup(params, arrays, tile=tile))
    assert len(set(tiles)) >= 2, tiles         # the cache picks different tiles by class
    plan = pic.Plan([m[0] for m in made], [m[3] for m in made], tune_cache=cache_path)
    assert plan.info()["blocks_per_cu"] == min(cache["blocks_per_cu"], plan.info()["blocks_per_cu"])
    Jb = pic.deposit_batched(plan, [m[2] for m in made], path="cell_valu")
    torch.cuda.synchronize()
    for k, ((params, arrays), (grid, og, parts, bins)) in enumerate(zip(patches, made)):
        Js = pic.deposit(grid, parts, bins, "cell_valu")
        torch.cuda.synchronize()
        for c in range(3):
            assert torch.equal(Jb[k][c], Js[c]), (k, c, tiles[k])
        want = oracle_J(og, arrays)
        assert max(rel_l2(Jb[k][c].cpu().numpy(), want[c]) for c in range(3)) <= TOL_FP32
    plan.close()
    for m in made:
        m[3].close()
