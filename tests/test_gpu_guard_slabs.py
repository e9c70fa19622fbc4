"""One-GPU check of the domain decomposition designed for several GPUs: a periodic grid
split into z-slabs, each slab deposited on its own in guard mode (Sec. 4.1 decomposes each
rank's domain into tiles; ranks own slabs), then every slab's guard planes added into the
planes of its neighbours (the exchange a multi-GPU run would do with send/recv). The sum
must equal the single periodic grid's J."""
import numpy as np
import pytest
import torch

from gpu_util import TOL_FP32, oracle_J, rel_l2, say, setup
from paper_2601_08277_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("order,nslab", [(3, 2), (1, 2), (2, 4)])
def test_guard_slabs_sum_to_periodic(order, nslab):
    say(f"case guard slabs order={order} nslab={nslab}")
    from paper_2601_08277_amd import pic
    n = (32, 32, 32)
    params, arrays = synth.uniform(3, n, 8, 0.05, order, seed=1002, dt=0.2)
    grid, og, parts, bins = setup(params, arrays, tile=(8, 8, 4))
    J_full = [j.cpu().numpy() for j in pic.deposit(grid, parts, bins, "cell_valu")]
    bins.close()
    ng = 3
    h = n[2] // nslab
    J_sum = [np.zeros((n[2], n[1], n[0]), np.float64) for _ in range(3)]
    for k in range(nslab):
        z0 = k * h
        sel = (arrays["z"] >= z0) & (arrays["z"] < z0 + h)
        sub = {name: np.ascontiguousarray(a[sel]) for name, a in arrays.items()}
        sp = dict(params, n=(n[0], n[1], h), bc=(0, 0, 1), ng=ng, x0=(0.0, 0.0, float(z0)))
        sg, _, sparts, sbins = setup(sp, sub, tile=(8, 8, 4))
        Js = pic.deposit(sg, sparts, sbins, "cell_valu")
        sbins.check()
        assert Js[0].shape == (h + 2 * ng, n[1], n[0])
        for c in range(3):
            a = Js[c].cpu().numpy().astype(np.float64)
            for m in range(h + 2 * ng):      # stored plane m is global node z0 + m - ng
                J_sum[c][(z0 + m - ng) % n[2]] += a[m]
        sbins.close()
    want = oracle_J(og, arrays)
    for c in range(3):
        assert rel_l2(J_sum[c], J_full[c]) <= TOL_FP32, c
        assert rel_l2(J_sum[c], want[c]) <= TOL_FP32, c
    torch.cuda.synchronize()
