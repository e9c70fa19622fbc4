"""Tile-shape, path and launch-shape autotuner for the deposition.

The paper fixes one tile size per run (Appendix A) and runs its matrix kernel where cells
are dense, vector kernels where they are sparse (Sec. 6.1, Sec. 7). On gfx950 both choices
are measured: for each (shape order, particles-per-cell bucket) the tuner times every
candidate tile on a synthetic guard-bounded patch of that class with each deposition path
(per-cell VALU, split-fp16 and split-bf16 MFMA, LDS-atomic), and keeps the fastest (tile,
path) among the paths that meet the float32 tolerance (the split-bf16 path, at about 4e-6,
does not and is only reported). It also times the persistent batched launch at each
feasible number of workgroups per compute unit. The result is a JSON cache:

    {"device": "...", "entries": [{"order": 3, "ppc": 8, "tile": [8, 8, 4],
                                   "path": "cell_valu", "ms": 0.41,
                                   "ms_paths": {"cell_valu": 0.41, "mfma_fp16": 2.3, ...}},
                                  ...],
     "blocks_per_cu": 3}

`lookup` picks the entry of the nearest ppc bucket for an order (tiles for the bins);
`pic_tuning_load` hands the same file to the library, whose PIC_PATH_AUTO then follows
the entries' paths by density; `pic_plan_create` reads "blocks_per_cu". Timing uses HIP
events on the current stream.
"""
import json
import math

import numpy as np

DEFAULT_TILES = [(8, 8, 4), (8, 8, 8), (4, 8, 8), (8, 4, 4), (4, 4, 4), (16, 8, 4), (8, 16, 4)]
DEFAULT_PPC = (2, 8, 32, 64)
PATHS = ("cell_valu", "mfma_fp16", "mfma_bf16", "atomic")
AUTO_PATHS = ("cell_valu", "mfma_fp16", "atomic")   # within the float32 tolerance


def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_tiles(orders=(1, 2, 3), ppcs=DEFAULT_PPC, tiles=DEFAULT_TILES, n=(48, 48, 48),
               reps=5, seed=0, paths=PATHS, log=None):
    """Fastest (tile, path) per (order, ppc) on a guard-bounded n-cell patch; every path's
    best time is kept in "ms_paths"."""
    from . import pic, synth
    entries = []
    for order in orders:
        for ppc in ppcs:
            params, arrays = synth.uniform(3, n, ppc, 0.05, order, seed=seed + 100 * order + ppc,
                                           bc=(1, 1, 1), ng=3)
            grid = pic.Grid(params)
            N = arrays["x"].size
            slots = pic.slots_for(N, int(np.prod(n)), 0.25)
            parts = pic.Particles.from_arrays(arrays, slots)
            J = pic.new_J(grid)
            best = {}          # path -> (ms, tile)
            for tile in tiles:
                try:
                    bins = pic.Bins(grid, tile, 0.25, slots)
                    pic.rebin(grid, parts, bins, pic.REBIN_FULL)
                except pic.PicError:
                    continue
                for path in paths:
                    try:
                        ms = _time(lambda: pic.deposit(grid, parts, bins, path, 0, J=J), reps)
                    except pic.PicError:
                        continue
                    if log:
                        log(f"order {order} ppc {ppc} tile {tile} {path}: {ms:.3f} ms")
                    if path not in best or ms < best[path][0]:
                        best[path] = (ms, tile)
                bins.close()
            elig = [p for p in AUTO_PATHS if p in best]
            if elig:
                win = min(elig, key=lambda p: best[p][0])
                entries.append({"order": order, "ppc": ppc, "tile": list(best[win][1]),
                                "path": win, "ms": best[win][0],
                                "ms_paths": {p: best[p][0] for p in best}})
    return entries


def tune_blocks(patches, entries, reps=5, log=None):
    """Fastest persistent workgroups per CU for a batched launch over `patches`
    ((params, arrays) pairs), with tiles from `entries`."""
    from . import pic
    grids, parts, bins = [], [], []
    for params, arrays in patches:
        g = pic.Grid(params)
        tile = lookup({"entries": entries}, params["order"], params.get("ppc", 8))[0]
        N = arrays["x"].size
        slots = pic.slots_for(N, int(np.prod(params["n"])), 0.25)
        p = pic.Particles.from_arrays(arrays, slots)
        b = pic.Bins(g, tile, 0.25, slots)
        pic.rebin(g, p, b, pic.REBIN_FULL)
        grids.append(g)
        parts.append(p)
        bins.append(b)
    plan = pic.Plan(grids, bins)
    occ = plan.info()["blocks_per_cu"]
    plan.close()
    best = None
    for bpc in range(1, occ + 1):
        path = _write_tmp({"blocks_per_cu": bpc})
        plan = pic.Plan(grids, bins, tune_cache=path)
        J = pic.deposit_batched(plan, parts)
        ms = _time(lambda: pic.deposit_batched(plan, parts, J), reps)
        plan.close()
        if log:
            log(f"blocks_per_cu {bpc}: {ms:.3f} ms")
        if best is None or ms < best[1]:
            best = (bpc, ms)
    for b in bins:
        b.close()
    return best[0]


def _write_tmp(obj):
    import tempfile
    f = tempfile.NamedTemporaryFile("w", suffix=".json", delete=False)
    json.dump(obj, f)
    f.close()
    return f.name


def tune(out_path, patches=None, log=None, **kw):
    """Run the tile search (and the launch-shape search when `patches` is given), write
    the cache to `out_path` and return it."""
    import torch
    cache = {"device": torch.cuda.get_device_name(0), "entries": tune_tiles(log=log, **kw)}
    if patches:
        cache["blocks_per_cu"] = tune_blocks(patches, cache["entries"], log=log)
    with open(out_path, "w") as f:
        json.dump(cache, f, indent=1)
    return cache


def load(path):
    with open(path) as f:
        return json.load(f)


def lookup(cache, order, ppc, default=(8, 8, 4)):
    """(tile, path) of the entry for `order` whose ppc bucket is nearest (log scale)."""
    best = None
    for e in cache.get("entries", []):
        if e["order"] != order:
            continue
        d = abs(math.log(max(ppc, 1e-3)) - math.log(max(e["ppc"], 1e-3)))
        if best is None or d < best[0]:
            best = (d, e)
    if best is None:
        return tuple(default), "cell_valu"
    return tuple(best[1]["tile"]), best[1]["path"]


def main():
    import argparse
    import os
    from . import synth
    ap = argparse.ArgumentParser(description="tune tiles and the batched launch shape")
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "tune_cache.json"))
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--batched-patches", type=int, default=16,
                    help="patches of the batched recipe (edges 32..64) for the launch shape; 0: skip")
    a = ap.parse_args()
    patches = None
    if a.batched_patches:
        patches = synth.c4_patches(npatch=a.batched_patches, edge=(32, 64), seed=2004)
    cache = tune(a.out, patches=patches, log=lambda m: print(m, flush=True), reps=a.reps)
    print(json.dumps(cache), flush=True)


if __name__ == "__main__":
    main()
