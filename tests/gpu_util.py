"""Helpers shared by the GPU parity tests (the oracle is called only from tests)."""
import sys

import numpy as np

from oracle import binning as ob
from oracle import deposit as od
from oracle.deposit import OracleGrid

TOL_FP32 = 1e-6     # rel-L2 per component against the FP64 oracle, float32 paths
TOL_SPLIT = 1e-5    # split bf16/fp16 MFMA paths


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(got, want):
    got = np.asarray(got, np.float64).ravel()
    want = np.asarray(want, np.float64).ravel()
    den = np.linalg.norm(want)
    return float(np.linalg.norm(got - want) / (den if den > 0 else 1.0))


def oracle_inputs(arrays, valid=None):
    pos = [arrays["x"], arrays["y"], arrays["z"]]
    u = [arrays["ux"], arrays["uy"], arrays["uz"]]
    return pos, u, arrays["w"]


def setup(params, arrays, tile=(8, 8, 8), slack=0.25, full=True, max_movers=0):
    """Grid, GPU particles, bins (after a FULL rebin) and the oracle grid."""
    from paper_2601_08277_amd import pic
    grid = pic.Grid(params)
    og = OracleGrid.from_params(params)
    N = arrays["x"].shape[0]
    ncell = int(np.prod(og.n))
    nslots = pic.slots_for(N, ncell, slack)
    parts = pic.Particles.from_arrays(arrays, nslots)
    t = tuple(tile[: params["dim"]]) + (1,) * (3 - params["dim"])
    bins = pic.Bins(grid, t, slack, nslots, max_movers)
    if full:
        pic.rebin(grid, parts, bins, pic.REBIN_FULL)
    return grid, og, parts, bins


def dense_slots(off, ln):
    """Slot index of every dense-prefix entry and the bin it belongs to."""
    total = int(ln.sum())
    b = np.repeat(np.arange(ln.size), ln)
    start = np.repeat(off[:-1].astype(np.int64), ln)
    first = np.repeat(np.cumsum(ln) - ln, ln)
    return start + (np.arange(total) - first), b


def check_bins(og, host, off, ln, bin_cell, ref_arrays=None, stale_ok=0):
    """Sorter invariants against the oracle. Returns the number of stale particles.

    host: particle arrays read back from the GPU. ref_arrays: arrays indexed by id whose
    payload must appear bitwise (the expected positions/momenta of every particle).
    """
    ids = host["id"]
    slots, b = dense_slots(off, ln)
    dense = np.zeros(ids.size, bool)
    dense[slots] = True
    assert np.all(ids[~dense] == -1), "a slot outside the dense prefixes holds a particle"
    assert np.all(host["w"][~dense] == 0), "a gap slot carries weight"
    assert np.all(ids[dense] != -1), "a gap inside a dense prefix"
    assert np.all(np.diff(off) >= ln), "len exceeds capacity"
    vid = ids[dense]
    assert np.unique(vid).size == vid.size, "an id appears twice"
    pos = [host["x"][slots], host["y"][slots], host["z"][slots]]
    cell = ob.cell_index(og, pos)
    stale = int(np.count_nonzero(cell != bin_cell[b]))
    assert stale <= stale_ok, f"{stale} particles sit in a bin of another cell"
    if ref_arrays is not None:
        assert vid.size == ref_arrays["id"].size, "particle count changed"
        order = np.argsort(vid)
        assert np.array_equal(vid[order], np.sort(ref_arrays["id"]))
        ref_index = np.empty(ref_arrays["id"].max() + 1, np.int64)
        ref_index[ref_arrays["id"]] = np.arange(ref_arrays["id"].size)
        k = ref_index[vid]
        for name in ("x", "y", "z", "ux", "uy", "uz", "w"):
            a = host[name][slots]
            r = ref_arrays[name][k]
            assert np.array_equal(a.view(np.uint8), r.astype(a.dtype).view(np.uint8)), \
                f"payload {name} not moved bitwise"
    if stale == 0:
        counts, sorted_ids, _ = ob.expected_bins(og, pos, vid, valid=np.ones(vid.size, bool))
        gpu_counts = np.zeros(int(np.prod(og.n)), np.int64)
        np.add.at(gpu_counts, bin_cell[b], 1)
        assert np.array_equal(gpu_counts, counts), "per-cell counts differ from the oracle"
        got = np.lexsort((vid, bin_cell[b]))
        assert np.array_equal(vid[got], sorted_ids), "per-cell id sets differ from the oracle"
    return stale


def oracle_J(og, arrays):
    pos, u, w = oracle_inputs(arrays)
    return od.deposit(og, pos, u, w)
