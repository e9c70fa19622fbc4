"""Pins of the binning oracle, the drift and the re-sort policy."""
import numpy as np
import pytest

from oracle import binning as ob
from oracle import deposit as od
from oracle.deposit import GUARD, PERIODIC, OracleGrid
from paper_2601_08277_amd import synth


def test_cell_index_matches_python_loop():
    g = OracleGrid(3, (5, 4, 3), 1)
    rng = np.random.default_rng(1)
    pos = [rng.uniform(0, g.n[d], 500) for d in range(3)]
    cell = ob.cell_index(g, pos)
    for p in range(500):
        i, j, k = (int(np.floor(pos[d][p])) for d in range(3))
        assert cell[p] == (k * 4 + j) * 5 + i


def test_cell_tie_breaks():
    g = OracleGrid(3, (4, 4, 4), 1)
    pos = [np.array([1.0, 4.0, np.nextafter(4.0, 0)]), np.array([0.0, 0.0, 0.0]), np.zeros(3)]
    cell = ob.cell_index(g, pos)
    assert list(cell) == [1, 3, 3]          # boundary -> upper cell, x == L -> clamped


def test_expected_bins_against_dict_of_sets():
    params, arr = synth.uniform(3, (6, 5, 4), 3, 0.1, 1, seed=3)
    g = OracleGrid.from_params(params)
    ids = arr["id"].copy()
    ids[::7] = -1                                         # some gap slots
    pos = [arr["x"], arr["y"], arr["z"]]
    counts, sorted_ids, cells = ob.expected_bins(g, pos, ids)
    ref = {}
    for p in range(ids.size):
        if ids[p] == -1:
            continue
        c = (int(arr["z"][p]) * 5 + int(arr["y"][p])) * 6 + int(arr["x"][p])
        ref.setdefault(c, []).append(int(ids[p]))
    assert counts.sum() == np.count_nonzero(ids != -1)
    for c in range(g.n[0] * g.n[1] * g.n[2]):
        assert counts[c] == len(ref.get(c, []))
    start = np.concatenate([[0], np.cumsum(counts)])
    for c, members in ref.items():
        assert list(sorted_ids[start[c]:start[c + 1]]) == sorted(members)
        assert np.all(cells[start[c]:start[c + 1]] == c)


def test_drift_periodic_wrap_and_mover_fraction():
    """Expected movers per step ~ dim * dt * sigma * sqrt(2/pi) for small sigma."""
    params, arr = synth.c1()
    g = OracleGrid.from_params(params)
    pos = [arr["x"], arr["y"], arr["z"]]
    u = [arr["ux"], arr["uy"], arr["uz"]]
    old = ob.cell_index(g, pos)
    new_pos = od.drift(g, pos, u, params["dt"])
    for d in range(2):
        assert np.all(new_pos[d] >= 0) and np.all(new_pos[d] <= g.n[d])
    np.testing.assert_array_equal(new_pos[2], pos[2])
    frac = ob.movers(g, new_pos, arr["id"], old) / arr["id"].size
    expect = 2 * params["dt"] * 0.01 * np.sqrt(2 / np.pi)
    assert abs(frac - expect) < 0.15 * expect


def test_drift_is_plain_kinematics():
    g = OracleGrid(3, (10, 10, 10), 1, bc=(PERIODIC, PERIODIC, GUARD), ng=2)
    pos = [np.array([9.9]), np.array([0.05]), np.array([5.0])]
    u = [np.array([0.75], np.float32), np.array([-0.75], np.float32), np.array([0.0], np.float32)]
    # gamma = sqrt(1 + 9/16 + 9/16) = sqrt(34)/4
    gam = np.sqrt(34.0) / 4.0
    out = od.drift(g, pos, u, 0.5)
    assert abs(out[0][0] - (9.9 + 0.75 / gam * 0.5 - 10.0)) < 1e-14
    assert abs(out[1][0] - (0.05 - 0.75 / gam * 0.5 + 10.0)) < 1e-14
    assert out[2][0] == 5.0


@pytest.mark.parametrize("case", [
    # steps, rebuilds, empty, perf, base  -> decision, trigger
    ((3, 500, 0.01, 0.1, 1.0), (False, 1)),     # min interval wins over everything
    ((50, 0, 0.25, None, None), (True, 2)),     # fixed interval
    ((20, 101, 0.25, None, None), (True, 3)),   # rebuilds exceed the count
    ((20, 100, 0.25, None, None), (False, 0)),  # equal is not exceeding
    ((20, 0, 0.10, None, None), (True, 4)),     # too few empty slots
    ((20, 0, 0.90, None, None), (True, 4)),     # too many empty slots
    ((20, 0, 0.25, 0.7, 1.0), (True, 5)),       # performance below 80 % of baseline
    ((20, 0, 0.25, 0.85, 1.0), (False, 0)),
    ((20, 0, None, None, None), (False, 0)),    # empty ratio not known yet: no trigger 4
    ((20, 101, None, None, None), (True, 3)),
    ((20, 0, None, 0.7, 1.0), (True, 5)),
])
def test_policy_truth_table(case):
    args, want = case
    steps, rebuilds, empty, perf, base = args
    assert ob.should_global_sort(steps, rebuilds, empty, perf, base) == want


def test_policy_perf_disabled():
    assert ob.should_global_sort(20, 0, 0.25, 0.1, 1.0, {"perf_enable": 0}) == (False, 0)
