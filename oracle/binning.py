"""What any correct cell sorter must produce, and the global re-sort policy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 4.1 (Alg. 1) keeps particles sorted by cell: a counting sort at start-up
(GlobalSortParticlesByCell), then per step only the particles whose cell changed are
moved (Sec. 4.3.1, stage 2: c_new != c_old marks a mover). Where a particle lands inside
its cell's bin is unspecified (the empty-slot stack hands out slots in pop order), so the
result that is unique is, per cell, the SET of particle ids and the COUNT. The oracle
gives those: a stable argsort by cell plus a bincount, with ids sorted inside each cell.

Cell index: the cell of each dimension from the deposition oracle's grid coordinate
(float64, floor, clamp of xi == n into n - 1), flattened x fastest:
    cell = (k * n_y + j) * n_x + i.

The policy (Sec. 4.4) evaluates five triggers in priority order after each step:
  1. fewer than min_interval steps since the last global sort -> no sort;
  2. at least `interval` steps since the last sort -> sort;
  3. local rebuilds since the last sort exceed rebuild_count -> sort;
  4. empty-slot ratio below empty_ratio or above full_ratio -> sort;
  5. (optional) performance below perf_degrad times the baseline -> sort.
Readings: trigger 4 compares the fraction of empty slots over all bins with both
thresholds (too full when below empty_ratio, too sparse when above full_ratio); the
baseline of trigger 5 is the performance of the first step after the last global sort,
higher meaning better. Defaults are the paper's parameter table (Appendix A). The policy
acts on the statistics known when it decides (Alg. 1 evaluates it on the step's collected
statistics): while no statistics of a step after the last global sort are known, the
empty-slot ratio is unknown (None) and trigger 4 cannot fire.
"""
import numpy as np

from .deposit import grid_coords

DEFAULT_POLICY = dict(min_interval=10, interval=50, rebuild_count=100,
                      empty_ratio=0.15, full_ratio=0.85, perf_enable=1, perf_degrad=0.80)


def cell_index(g, pos):
    """Flat x-fastest cell of every particle (int64)."""
    _, cells = grid_coords(g, pos[: g.dim])
    flat = cells[g.dim - 1]
    for d in reversed(range(g.dim - 1)):
        flat = flat * g.n[d] + cells[d]
    return flat


def n_cells(g):
    return int(np.prod(g.n))


def expected_bins(g, pos, ids, valid=None):
    """Canonical binning: (counts per cell, ids sorted by (cell, id), cell of each).

    counts[c] = number of valid particles in cell c; the second array lists every valid
    id, grouped by cell in increasing cell order and increasing id inside a cell.
    """
    ids = np.asarray(ids)
    if valid is None:
        valid = ids != -1
    pos = [np.asarray(p)[valid] for p in pos[: g.dim]]
    ids = ids[valid]
    cell = cell_index(g, pos)
    counts = np.bincount(cell, minlength=n_cells(g))
    order = np.lexsort((ids, cell))
    return counts, ids[order], cell[order]


def movers(g, pos, ids, old_cell, valid=None):
    """Number of valid particles whose cell differs from the cell of their old bin."""
    ids = np.asarray(ids)
    if valid is None:
        valid = ids != -1
    new_cell = cell_index(g, [np.asarray(p)[valid] for p in pos[: g.dim]])
    return int(np.count_nonzero(new_cell != np.asarray(old_cell)[valid]))


def should_global_sort(steps_since_sort, rebuilds_since_sort, empty_slot_ratio,
                       perf=None, perf_baseline=None, policy=None):
    """Return (decision, trigger number or 0) following the prioritised list above."""
    p = dict(DEFAULT_POLICY)
    if policy:
        p.update(policy)
    if steps_since_sort < p["min_interval"]:
        return False, 1
    if steps_since_sort >= p["interval"]:
        return True, 2
    if rebuilds_since_sort > p["rebuild_count"]:
        return True, 3
    if empty_slot_ratio is not None and (empty_slot_ratio < p["empty_ratio"]
                                         or empty_slot_ratio > p["full_ratio"]):
        return True, 4
    if (p["perf_enable"] and perf is not None and perf_baseline is not None
            and perf < p["perf_degrad"] * perf_baseline):
        return True, 5
    return False, 0
