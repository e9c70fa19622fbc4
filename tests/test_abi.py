"""CPU checks of the C ABI: the library loads, exports every function pic.h declares, the
host-side policy agrees with the oracle, and argument errors are reported without a GPU."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

from oracle import binning as ob

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic.h")
LIB = os.path.join(ROOT, "paper_2601_08277_amd", "libpic.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(pic_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.fail("libpic.so is not built (run __graft_entry__.build())")
    from paper_2601_08277_amd import pic
    return pic.lib()


def test_header_declares_core_calls():
    names = declared_functions()
    for must in ("pic_deposit", "pic_rebin", "pic_deposit_backward", "pic_bins_create",
                 "pic_deposit_batched", "pic_plan_create"):
        assert must in names


def test_every_declared_symbol_is_exported(L):
    for name in declared_functions():
        assert hasattr(L, name), f"{name} declared in pic.h but not exported"


def test_binding_lists_every_symbol():
    from paper_2601_08277_amd import pic
    assert sorted(pic.EXPORTS) == declared_functions()


@pytest.mark.parametrize("case", [
    (3, 500, 0.01, 0.1, 1.0), (50, 0, 0.25, 0.0, 0.0), (20, 101, 0.25, 0.0, 0.0),
    (20, 100, 0.25, 0.0, 0.0), (20, 0, 0.10, 0.0, 0.0), (20, 0, 0.90, 0.0, 0.0),
    (20, 0, 0.25, 0.7, 1.0), (20, 0, 0.25, 0.85, 1.0), (10, 0, 0.5, 0.0, 0.0),
    (49, 0, 0.15, 0.0, 0.0), (49, 0, 0.85, 0.0, 0.0), (20, 0, -1.0, 0.0, 0.0),
    (20, 101, -1.0, 0.0, 0.0)])
def test_policy_matches_oracle(L, case):
    from paper_2601_08277_amd import pic
    steps, reb, empty, perf, base = case
    want = ob.should_global_sort(steps, reb, empty if empty >= 0 else None,
                                 perf if perf > 0 else None, base if base > 0 else None)
    assert pic.policy_decide(steps, reb, empty, perf, base) == want


def test_policy_random_agreement(L):
    from paper_2601_08277_amd import pic
    rng = np.random.default_rng(0)
    pol = pic.policy(min_interval=5, interval=30, rebuild_count=7, empty_ratio=0.2,
                     full_ratio=0.7, perf_enable=1, perf_degrad=0.9)
    pd = dict(min_interval=5, interval=30, rebuild_count=7, empty_ratio=0.2, full_ratio=0.7,
              perf_enable=1, perf_degrad=0.9)
    for _ in range(500):
        steps = int(rng.integers(0, 40))
        reb = int(rng.integers(0, 12))
        empty = float(rng.uniform(0, 1))
        perf, base = float(rng.uniform(0.5, 1.5)), float(rng.uniform(0.5, 1.5))
        want = ob.should_global_sort(steps, reb, empty, perf, base, pd)
        assert pic.policy_decide(steps, reb, empty, perf, base, pol) == want


def test_argument_errors_without_gpu(L):
    from paper_2601_08277_amd import pic
    g = pic.PicGrid()
    g.dim = 4
    h = ctypes.c_void_p()
    t = (ctypes.c_int * 3)(8, 8, 8)
    st = L.pic_bins_create(ctypes.byref(g), t, 0.25, 100, 0, ctypes.byref(h))
    assert st == -1 and b"dim" in L.pic_last_error()
    g.dim = 3
    for d in range(3):
        g.n[d] = 8
        g.dx[d] = 1.0
        g.inv_dx[d] = 1.0
        g.bc[d] = 1
    g.order = 3
    g.ng = 1                      # order 3 needs 2 guard nodes
    st = L.pic_bins_create(ctypes.byref(g), t, 0.25, 100, 0, ctypes.byref(h))
    assert st == -1 and b"ng" in L.pic_last_error()
    assert L.pic_deposit(None, None, None, None, None, None, 0, 0, None) == -1


def _grid3(pic, order=3, dt=0.5):
    g = pic.PicGrid()
    g.dim = 3
    for d in range(3):
        g.n[d] = 8
        g.dx[d] = 1.0
        g.inv_dx[d] = 1.0
        g.bc[d] = 0
    g.order = order
    g.q = -1.0
    g.dt = dt
    return g


def _fake_particles(pic, n=16):
    """Descriptor with non-NULL but never-dereferenced pointers: every check below fails
    before anything is launched."""
    p = pic.PicParticles()
    p.nslots = n
    for name in ("x", "y", "z", "ux", "uy", "uz", "w", "id"):
        setattr(p, name, 4096)
    return p


def test_argument_errors_of_the_next_rows_without_gpu(L):
    from paper_2601_08277_amd import pic
    g = _grid3(pic)
    p = _fake_particles(pic)
    f = ctypes.c_void_p(4096)
    # push: flags must be 0, qm and dt finite
    assert L.pic_push(ctypes.byref(g), ctypes.byref(p), None, *[f] * 6, -1.0, 0.2, 1, None) == -1
    assert b"flags" in L.pic_last_error()
    assert L.pic_push(ctypes.byref(g), ctypes.byref(p), None, *[f] * 6, float("nan"), 0.2, 0,
                      None) == -1
    assert L.pic_push(ctypes.byref(g), ctypes.byref(p), None, None, *[f] * 5, -1.0, 0.2, 0,
                      None) == -1
    # Esirkepov: dt must be non-zero, ACCUMULATE is the only flag, old positions needed
    g0 = _grid3(pic, dt=0.0)
    assert L.pic_deposit_esirkepov(ctypes.byref(g0), ctypes.byref(p), None, f, f, f, f, f, f, 0,
                                   None) == -1
    assert b"dt" in L.pic_last_error()
    assert L.pic_deposit_esirkepov(ctypes.byref(g), ctypes.byref(p), None, f, f, f, f, f, f,
                                   pic.F_DRIFT, None) == -1
    assert L.pic_deposit_esirkepov(ctypes.byref(g), ctypes.byref(p), None, None, f, f, f, f, f,
                                   0, None) == -1
    assert b"old" in L.pic_last_error()
    # midpoint: refused on the tile-atomic and MFMA paths before bins are looked at
    for path in (pic.PATH_NAMES["atomic"], pic.PATH_NAMES["mfma_bf16"]):
        assert L.pic_deposit(ctypes.byref(g), ctypes.byref(p), None, f, f, f, path,
                             pic.F_MIDPOINT, None) == pic.PIC_ERR_UNSUPPORTED
    # charge density takes ACCUMULATE only; gather needs every pointer
    assert L.pic_deposit_rho(ctypes.byref(g), ctypes.byref(p), None, f, pic.F_DRIFT, None) == -1
    assert L.pic_gather_fields(ctypes.byref(g), ctypes.byref(p), None, *[f] * 11, None,
                               None) == -1


def test_tuning_cache_parser(L, tmp_path):
    """pic_tuning_load reads the autotuner's cache (nested "tile" lists and "ms_paths"
    objects included) and rejects malformed or unknown entries; no GPU needed."""
    from paper_2601_08277_amd import pic
    committed = os.path.join(ROOT, "paper_2601_08277_amd", "tune_cache.json")
    assert L.pic_tuning_load(committed.encode()) == pic.PIC_OK
    good = tmp_path / "good.json"
    good.write_text(json.dumps({"device": "x", "entries": [
        {"order": 3, "ppc": 8, "tile": [8, 8, 4], "path": "mfma_fp16", "ms": 1.0,
         "ms_paths": {"cell_valu": 0.5, "mfma_fp16": 1.0, "path": 3}},
        {"order": 1, "ppc": 2, "tile": [8, 4, 4], "path": "cell_valu", "ms": 0.1}],
        "blocks_per_cu": 2}))
    assert L.pic_tuning_load(str(good).encode()) == pic.PIC_OK
    for bad in ({"entries": [{"order": 3, "ppc": 8, "path": "fastest"}]},
                {"entries": [{"order": 4, "ppc": 8, "path": "cell_valu"}]},
                {"entries": [{"order": 3, "path": "cell_valu"}]},
                {"no_entries": []}):
        f = tmp_path / "bad.json"
        f.write_text(json.dumps(bad))
        assert L.pic_tuning_load(str(f).encode()) == pic.PIC_ERR_INVALID_ARG, bad
    f = tmp_path / "trunc.json"
    f.write_text(json.dumps({"entries": [{"order": 3, "ppc": 8, "path": "cell_valu"}]})[:-3])
    assert L.pic_tuning_load(str(f).encode()) == pic.PIC_ERR_INVALID_ARG
    assert L.pic_tuning_load(str(tmp_path / "missing.json").encode()) == pic.PIC_ERR_INVALID_ARG
    assert L.pic_tuning_load(None) == pic.PIC_OK


def test_unused_flag_bit_is_rejected_without_gpu(L):
    """Flag bit 2 has no meaning (the bins are always kept in a deterministic order and the
    repeatability of J depends on the path, see pic.h): every call that takes flags
    rejects it before looking at bins or launching anything."""
    from paper_2601_08277_amd import pic
    g = _grid3(pic)
    p = _fake_particles(pic)
    f = ctypes.c_void_p(4096)
    for path in (pic.PATH_CELL_VALU, pic.PATH_UNSORTED):
        assert L.pic_deposit(ctypes.byref(g), ctypes.byref(p), None, f, f, f, path, 2,
                             None) == pic.PIC_ERR_INVALID_ARG
        assert b"flag" in L.pic_last_error()
        assert L.pic_deposit_noalloc(ctypes.byref(g), ctypes.byref(p), None, f, f, f, path, 2,
                                     None) == pic.PIC_ERR_INVALID_ARG
    assert L.pic_deposit_rho(ctypes.byref(g), ctypes.byref(p), None, f, 2, None) == -1
    assert L.pic_deposit_backward(ctypes.byref(g), ctypes.byref(p), None, f, f, f, f, f, f, f,
                                  f, f, None, 2, None) == -1
    assert b"flags" in L.pic_last_error()
