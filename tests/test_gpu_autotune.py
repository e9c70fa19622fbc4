"""The autotuner on the GPU and PIC_PATH_AUTO following its cache (density-based choice
between the per-cell VALU path and the matrix paths, Sec. 6.1 / Sec. 7), on single grids
and in a batched plan, against the FP64 oracle."""
import json

import numpy as np
import pytest
import torch

from gpu_util import TOL_FP32, TOL_SPLIT, oracle_J, rel_l2, say, setup
from paper_2601_08277_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture
def clean_tuning():
    from paper_2601_08277_amd import pic
    pic.tuning_load(None)
    yield
    pic.tuning_load(None)


def test_tune_tiles_small(clean_tuning, tmp_path):
    """A small tuning run: one entry per (order, ppc), the fastest path within the float32
    tolerance, every path timed, and the library accepts the cache it writes."""
    say("case tune_tiles small")
    from paper_2601_08277_amd import autotune, pic
    tiles = [(8, 8, 4), (4, 4, 4)]
    entries = autotune.tune_tiles(orders=(1, 3), ppcs=(4, 16), tiles=tiles, n=(20, 20, 16),
                                  reps=2)
    assert [(e["order"], e["ppc"]) for e in entries] == [(1, 4), (1, 16), (3, 4), (3, 16)]
    for e in entries:
        assert tuple(e["tile"]) in tiles
        assert e["path"] in autotune.AUTO_PATHS
        assert set(e["ms_paths"]) == set(autotune.PATHS)
        assert all(v > 0 for v in e["ms_paths"].values())
        assert e["ms"] == min(e["ms_paths"][p] for p in autotune.AUTO_PATHS)
    f = tmp_path / "cache.json"
    f.write_text(json.dumps({"device": "test", "entries": entries}))
    pic.tuning_load(str(f))


def _forced_cache(tmp_path, rows):
    f = tmp_path / "forced.json"
    f.write_text(json.dumps({"entries": [
        {"order": o, "ppc": p, "tile": [8, 8, 4], "path": path} for o, p, path in rows]}))
    return str(f)


def test_auto_follows_cache_by_density(clean_tuning, tmp_path):
    """A cache that puts order 3 at 8 per cell on the split-fp16 matrix path and order 3 at
    48 per cell on the VALU path: AUTO picks by the bins' density, runs that path (J equal
    to the named path's), matches the oracle, and returns to VALU when the cache is
    cleared."""
    from paper_2601_08277_amd import pic
    pic.tuning_load(_forced_cache(tmp_path, [(3, 8, "mfma_fp16"), (3, 48, "cell_valu")]))
    for ppc, want_path, tol in ((8, "mfma_fp16", TOL_SPLIT), (40, "cell_valu", TOL_FP32)):
        say(f"case auto cache ppc={ppc}")
        params, arrays = synth.uniform(3, (20, 18, 16), ppc, 0.05, 3, seed=50 + ppc)
        grid, og, parts, bins = setup(params, arrays, tile=(8, 8, 4))
        assert pic.auto_path(grid, bins) == want_path
        J_auto = pic.deposit(grid, parts, bins, "auto")
        J_named = pic.deposit(grid, parts, bins, want_path)
        torch.cuda.synchronize()
        want = oracle_J(og, arrays)
        for c in range(3):
            a = J_auto[c].cpu().numpy()
            assert np.array_equal(a, J_named[c].cpu().numpy()), (ppc, c)
            assert rel_l2(a, want[c]) <= tol, (ppc, c, rel_l2(a, want[c]))
        pic.tuning_load(None)
        assert pic.auto_path(grid, bins) == "cell_valu"
        pic.tuning_load(_forced_cache(tmp_path, [(3, 8, "mfma_fp16"), (3, 48, "cell_valu")]))
        bins.close()


def test_batched_plan_honours_cache(clean_tuning, tmp_path):
    """Patches of order 2 go to the split-fp16 matrix path by the cache, the others stay on
    the per-cell path; one batched AUTO call deposits all of them, each within its path's
    tolerance of the oracle; with PIC_PATH_CELL_VALU every patch runs on the per-cell path."""
    say("case batched honours cache")
    from paper_2601_08277_amd import pic
    pic.tuning_load(_forced_cache(tmp_path, [(2, 8, "mfma_fp16"), (1, 8, "cell_valu"),
                                             (3, 8, "cell_valu")]))
    shapes = [((20, 16, 12), 1), ((16, 16, 16), 2), ((12, 20, 16), 3), ((18, 14, 12), 2)]
    grids, parts, bins, ogs, arrs = [], [], [], [], []
    for k, (n, order) in enumerate(shapes):
        params, arrays = synth.uniform(3, n, 6, 0.05, order, seed=60 + k, bc=(1, 1, 1), ng=3)
        g, og, p, b = setup(params, arrays, tile=(8, 8, 4))
        grids.append(g)
        parts.append(p)
        bins.append(b)
        ogs.append(og)
        arrs.append(arrays)
    plan = pic.Plan(grids, bins)
    paths = [plan.patch_path(k) for k in range(len(shapes))]
    assert paths == ["cell_valu", "mfma_fp16", "cell_valu", "mfma_fp16"]
    for mode in ("auto", "cell_valu"):
        Js = pic.deposit_batched(plan, parts, path=mode)
        torch.cuda.synchronize()
        for k in range(len(shapes)):
            want = oracle_J(ogs[k], arrs[k])
            tol = TOL_SPLIT if (mode == "auto" and paths[k] != "cell_valu") else TOL_FP32
            ref = pic.deposit(grids[k], parts[k], bins[k], paths[k] if mode == "auto" else "cell_valu")
            torch.cuda.synchronize()
            for c in range(3):
                a = Js[k][c].cpu().numpy()
                assert rel_l2(a, want[c]) <= tol, (mode, k, c)
                assert rel_l2(a, ref[c].cpu().numpy()) <= tol, (mode, k, c)
    plan.close()
    for b in bins:
        b.check()
        b.close()
