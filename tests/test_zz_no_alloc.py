"""pic_deposit_noalloc (tile windows in the library's fixed device array) against
pic_deposit and the FP64 oracle, through the C ABI: two calls in a row, the second on a
smaller grid, and the refusal of bins whose windows exceed the array."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import TOL_FP32, oracle_J, rel_l2, say, setup
from paper_2601_08277_amd import synth

pytestmark = pytest.mark.gpu


def _noalloc(pic, grid, parts, bins, path, flags=0):
    J = pic.new_J(grid)
    pc = parts.c()
    st = pic.lib().pic_deposit_noalloc(ctypes.byref(grid.c), ctypes.byref(pc), bins.h,
                                       J[0].data_ptr(), J[1].data_ptr(), J[2].data_ptr(),
                                       pic.PATH_NAMES[path], flags,
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == pic.PIC_OK, pic.lib().pic_last_error()
    return J


@pytest.mark.parametrize("path", ["cell_valu", "atomic"])
def test_noalloc_matches_deposit(path):
    from paper_2601_08277_amd import pic
    cases = [((40, 36, 44), 8, 3, (8, 8, 4)), ((20, 17, 12), 5, 2, (8, 8, 4))]
    for n, ppc, order, tile in cases:      # the second call is smaller
        say(f"case noalloc {path} n={n} order={order}")
        params, arrays = synth.uniform(3, n, ppc, 0.05, order, seed=77 + order)
        grid, og, parts, bins = setup(params, arrays, tile=tile)
        J_na = _noalloc(pic, grid, parts, bins, path)
        J_ref = pic.deposit(grid, parts, bins, path)
        torch.cuda.synchronize()
        want = oracle_J(og, arrays)
        for c in range(3):
            a = J_na[c].cpu().numpy()
            assert rel_l2(a, J_ref[c].cpu().numpy()) <= TOL_FP32, (n, c)
            assert rel_l2(a, want[c]) <= TOL_FP32, (n, c)
        bins.check()
        bins.close()


def test_noalloc_refuses_large_windows():
    """128^3 cells in 8x8x4 tiles need 113 MB of windows: refused before any launch."""
    say("case noalloc refusal")
    from paper_2601_08277_amd import pic
    params = synth._params(3, (128, 128, 128), 3, dt=0.2)
    grid = pic.Grid(params)
    parts = pic.Particles(1024)
    bins = pic.Bins(grid, (8, 8, 4), 0.25, 1024)
    pic.rebin(grid, parts, bins, pic.REBIN_FULL)
    J = pic.new_J(grid)
    pc = parts.c()
    st = pic.lib().pic_deposit_noalloc(ctypes.byref(grid.c), ctypes.byref(pc), bins.h,
                                       J[0].data_ptr(), J[1].data_ptr(), J[2].data_ptr(),
                                       pic.PATH_CELL_VALU, 0,
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == pic.PIC_ERR_INVALID_ARG
    assert b"scratch" in pic.lib().pic_last_error()
    bins.check()
    bins.close()
