"""GPU parity of pic_deposit_backward against the oracle adjoint and FP64 central
differences, and of the torch.autograd wrapper."""
import numpy as np
import pytest
import torch

from gpu_util import TOL_FP32, oracle_inputs, rel_l2, say, setup
from oracle import deposit as od
from paper_2601_08277_amd import synth

pytestmark = pytest.mark.gpu

NAMES = ("dx", "dy", "dz", "dux", "duy", "duz", "dw")


def _grads(grid, parts, bins, G):
    from paper_2601_08277_amd import pic
    out = pic.deposit_backward(grid, parts, bins, [torch.from_numpy(g).cuda() for g in G])
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


@pytest.mark.parametrize("name,make", [
    ("c5-scaled-24^3-o3", lambda: synth.c5(n=(24, 24, 24))),
    ("o1-guard", lambda: synth.uniform(3, (12, 10, 9), 4, 0.3, 1, seed=3, bc=(1, 1, 1), ng=2)),
    ("o2-periodic", lambda: synth.uniform(3, (11, 13, 10), 4, 0.3, 2, seed=4)),
    ("2d-o3", lambda: synth.uniform(2, (20, 18), 6, 0.3, 3, seed=5)),
])
def test_backward_matches_oracle_adjoint(name, make):
    say(f"case backward {name}")
    params, arrays = make()
    grid, og, parts, bins = setup(params, arrays)
    G = synth.adjoint_field(grid.shape)
    got = _grads(grid, parts, bins, G)
    # gradients are per slot: map slots -> ids
    ids = parts.id.cpu().numpy()
    valid = ids != -1
    order = np.argsort(ids[valid])
    pos, u, w = oracle_inputs(arrays)
    want = od.deposit_adjoint(og, pos, u, w, [g.astype(np.float64) for g in G])
    for k in NAMES:
        if k == "dz" and params["dim"] == 2:
            continue
        gk = got[k][valid][order]
        assert rel_l2(gk, want[k]) <= TOL_FP32, (k, rel_l2(gk, want[k]))
        assert np.all(got[k][~valid] == 0)
    bins.close()


def test_c5_full_size_sampled_fd_and_autograd():
    """64^3, 8 per cell, order 3: autograd of L = sum J.G against FP64 central
    differences and the oracle adjoint on 1000 sampled particles."""
    say("case c5 full size")
    from paper_2601_08277_amd import pic
    params, arrays = synth.c5()
    grid, og, parts, bins = setup(params, arrays)
    G = synth.adjoint_field(grid.shape)
    Gt = [torch.from_numpy(g).cuda() for g in G]
    for name in ("x", "y", "z", "ux", "uy", "uz", "w"):
        getattr(parts, name).requires_grad_(True)
    J = pic.deposit_autograd(grid, parts, bins, pic.PATH_ATOMIC)
    L = sum((J[c] * Gt[c]).sum() for c in range(3))
    L.backward()
    torch.cuda.synchronize()
    grads = {k: getattr(parts, k[1:] if k != "dw" else "w").grad.detach().cpu().numpy()
             for k in ("dx", "dy", "dz", "dux", "duy", "duz", "dw")}
    ids = parts.id.detach().cpu().numpy()
    slot_of = np.empty(arrays["id"].size, np.int64)
    slot_of[ids[ids != -1]] = np.flatnonzero(ids != -1)
    sample = synth.sample_indices(arrays["id"].size, 1000, seed=1005)
    sub = {k: v[sample] for k, v in arrays.items()}
    pos, u, w = oracle_inputs(sub)
    Gd = [g.astype(np.float64) for g in G]
    want = od.deposit_adjoint(og, pos, u, w, Gd)
    for k in NAMES:
        gk = grads[k][slot_of[sub["id"]]]
        assert rel_l2(gk, want[k]) <= TOL_FP32, (k, rel_l2(gk, want[k]))
    # FP64 central differences of the particle's own contribution L_p = sum_c <G_c, J_c^(p)>
    h = 1e-6
    fd = {k: np.zeros(len(sample)) for k in ("dx", "dy", "dz", "dux")}
    for i in range(len(sample)):
        P = [np.array([pos[d][i]]) for d in range(3)]
        U = [np.array([np.float64(u[c][i])]) for c in range(3)]
        W = np.array([np.float64(w[i])])

        def Lp(P_, U_):
            Jp = od.deposit(og, P_, U_, W)
            return sum(float((Jp[c] * Gd[c]).sum()) for c in range(3))

        for d, k in enumerate(("dx", "dy", "dz")):
            Pp = [a.copy() for a in P]
            Pm = [a.copy() for a in P]
            Pp[d] += h
            Pm[d] -= h
            fd[k][i] = (Lp(Pp, U) - Lp(Pm, U)) / (2 * h)
        Up = [a.copy() for a in U]
        Um = [a.copy() for a in U]
        Up[0] += h
        Um[0] -= h
        fd["dux"][i] = (Lp(P, Up) - Lp(P, Um)) / (2 * h)
    for k, v in fd.items():
        gk = grads[k][slot_of[sub["id"]]]
        assert rel_l2(gk, v) <= 1e-5, (k, rel_l2(gk, v))
    bins.close()


@pytest.mark.parametrize("with_bins", [True, False])
def test_backward_with_stale_bins_and_without_bins(with_bins):
    """Particles left in the bins of other cells (every insert overflows at slack 0) take
    the listed global-gather path of the tiled kernel; without bins the particle-parallel
    kernel runs. Both against the oracle adjoint at the moved positions."""
    from paper_2601_08277_amd import pic
    say(f"case backward stale bins={with_bins}")
    params, arrays = synth.uniform(3, (16, 12, 12), 4, 0.4, 3, seed=21)
    grid, og, parts, bins = setup(params, arrays, tile=(4, 4, 4), slack=0.0)
    pic.drift(grid, parts, 1.5)
    pic.rebin(grid, parts, bins, pic.REBIN_INCREMENTAL)
    st = bins.stats()
    assert st["n_overflow"] > 0
    G = synth.adjoint_field(grid.shape)
    got = _grads(grid, parts, bins if with_bins else None, G)
    host = parts.to_numpy()
    valid = host["id"] != -1
    sub = {k: v[valid] for k, v in host.items()}
    pos, u, w = oracle_inputs(sub)
    want = od.deposit_adjoint(og, pos, u, w, [g.astype(np.float64) for g in G])
    for k in NAMES:
        assert rel_l2(got[k][valid], want[k]) <= TOL_FP32, (k, rel_l2(got[k][valid], want[k]))
        assert np.all(got[k][~valid] == 0)
    bins.check()
    bins.close()


def test_autograd_refuses_moved_particles():
    """The backward recomputes weights from the particles as they are when it runs, so a
    rebin (or any move) between forward and backward must raise instead of returning
    gradients of other positions; without a move the backward runs."""
    say("case autograd stale particles")
    from paper_2601_08277_amd import pic
    params, arrays = synth.c2(n=(16, 16, 16))
    grid, og, parts, bins = setup(params, arrays)
    G = [torch.from_numpy(g).cuda() for g in synth.adjoint_field(grid.shape)]
    parts.x.requires_grad_(True)
    J = pic.deposit_autograd(grid, parts, bins, pic.PATH_CELL_VALU)
    loss = sum((J[c] * G[c]).sum() for c in range(3))
    loss.backward()
    assert parts.x.grad is not None
    parts.x.grad = None
    J = pic.deposit_autograd(grid, parts, bins, pic.PATH_CELL_VALU)
    loss = sum((J[c] * G[c]).sum() for c in range(3))
    pic.drift(grid, parts, params["dt"])
    with pytest.raises(RuntimeError, match="moved or changed"):
        loss.backward()
    parts.x.requires_grad_(False)
    bins.close()
