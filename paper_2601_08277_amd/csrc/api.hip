// Host side of the libpic C ABI: argument validation, bins lifetime, dispatch and the
// global re-sort policy (Sec. 4.4). Kernels live in deposit.hip, rebin.hip, backward.hip.
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "pic_host.h"
#include "deposit_common.h"

static thread_local std::string g_last_error;

pic_status set_error(pic_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

pic_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return PIC_OK;
  return set_error(PIC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                                   \
  do {                                                  \
    pic_status _st = check_hip((call), #call);          \
    if (_st != PIC_OK) return _st;                      \
  } while (0)

extern "C" const char* pic_last_error(void) { return g_last_error.c_str(); }

// ----------------------------------------------------------------------------------
static int min_guard(int order) { return order == 1 ? 1 : 2; }

pic_status validate_grid(const pic_grid* g) {
  if (!g) return set_error(PIC_ERR_INVALID_ARG, "grid is NULL");
  if (g->dim != 2 && g->dim != 3) return set_error(PIC_ERR_INVALID_ARG, "dim must be 2 or 3");
  if (g->order < 1 || g->order > 3)
    return set_error(PIC_ERR_INVALID_ARG, "order must be 1, 2 or 3");
  if (g->dim == 2 && g->n[2] != 1)
    return set_error(PIC_ERR_INVALID_ARG, "2D grids need n[2] == 1");
  int64_t total = 1;
  for (int d = 0; d < g->dim; ++d) {
    if (g->n[d] < 1) return set_error(PIC_ERR_INVALID_ARG, "n must be positive");
    if (!(g->dx[d] > 0.0) || !(g->inv_dx[d] > 0.0) || !std::isfinite(g->inv_dx[d]) ||
        !std::isfinite(g->x0[d]))
      return set_error(PIC_ERR_INVALID_ARG, "dx, inv_dx must be positive and finite");
    if (g->bc[d] != PIC_BC_PERIODIC && g->bc[d] != PIC_BC_GUARD)
      return set_error(PIC_ERR_INVALID_ARG, "bc must be PIC_BC_PERIODIC or PIC_BC_GUARD");
    if (g->bc[d] == PIC_BC_PERIODIC && g->n[d] < 3)
      return set_error(PIC_ERR_INVALID_ARG, "periodic dimensions need n >= 3");
    if (g->bc[d] == PIC_BC_GUARD && g->ng < min_guard(g->order))
      return set_error(PIC_ERR_INVALID_ARG, "ng too small for this order (1, 2, 2 for orders 1-3)");
    int64_t N = g->n[d] + (g->bc[d] == PIC_BC_GUARD ? 2 * (int64_t)g->ng : 0);
    total *= N;
  }
  if (total >= (1ll << 31)) return set_error(PIC_ERR_INVALID_ARG, "grid has 2^31 or more nodes");
  return PIC_OK;
}

pic_status validate_particles(const pic_particles* p, int dim) {
  if (!p) return set_error(PIC_ERR_INVALID_ARG, "particles is NULL");
  if (p->nslots < 0 || p->nslots >= (1ll << 31) - 64)
    return set_error(PIC_ERR_INVALID_ARG, "nslots must be in [0, 2^31 - 64)");
  if (p->nslots > 0 && (!p->x || !p->y || (dim == 3 && !p->z) || !p->ux || !p->uy || !p->uz ||
                        !p->w || !p->id))
    return set_error(PIC_ERR_INVALID_ARG, "particle array pointer is NULL");
  return PIC_OK;
}

bool same_grid(const pic_grid& a, const pic_grid& b) {
  if (a.dim != b.dim) return false;
  for (int d = 0; d < 3; ++d)
    if (a.n[d] != b.n[d]) return false;
  return true;
}

KGrid make_kgrid(const pic_grid& g) {
  KGrid k{};
  k.dim = g.dim;
  k.order = g.order;
  for (int d = 0; d < 3; ++d) {
    bool used = d < g.dim;
    k.n[d] = used ? g.n[d] : 1;
    k.per[d] = used ? (g.bc[d] == PIC_BC_PERIODIC) : 1;
    k.g[d] = (used && !k.per[d]) ? g.ng : 0;
    k.N[d] = k.n[d] + 2 * k.g[d];
    k.x0[d] = used ? g.x0[d] : 0.0;
    k.inv_dx[d] = used ? g.inv_dx[d] : 1.0;
    k.inv_dxf[d] = (float)k.inv_dx[d];
    k.L[d] = used ? (double)g.n[d] * g.dx[d] : 1.0;
  }
  k.q = g.q;
  return k;
}

KPart make_kpart(const pic_particles& p) {
  KPart k{};
  k.x = p.x;
  k.y = p.y;
  k.z = p.z ? p.z : p.x;
  k.ux = p.ux;
  k.uy = p.uy;
  k.uz = p.uz;
  k.w = p.w;
  k.id = p.id;
  k.nslots = (int32_t)p.nslots;
  return k;
}

// ----------------------------------------------------------------------------------
extern "C" void pic_sort_policy_default(pic_sort_policy* out) {
  if (!out) return;
  out->min_interval = 10;
  out->interval = 50;
  out->rebuild_count = 100;
  out->empty_ratio = 0.15;
  out->full_ratio = 0.85;
  out->perf_enable = 1;
  out->perf_degrad = 0.80;
}

extern "C" int pic_policy_decide(const pic_sort_policy* p, int steps_since_sort,
                                 int rebuilds_since_sort, double empty_slot_ratio, double perf,
                                 double perf_baseline, int* trigger) {
  pic_sort_policy d;
  pic_sort_policy_default(&d);
  if (!p) p = &d;
  int t = 0, decide = 0;
  if (steps_since_sort < p->min_interval) {
    t = 1;
    decide = 0;
  } else if (steps_since_sort >= p->interval) {
    t = 2;
    decide = 1;
  } else if (rebuilds_since_sort > p->rebuild_count) {
    t = 3;
    decide = 1;
  } else if (empty_slot_ratio >= 0.0 &&
             (empty_slot_ratio < p->empty_ratio || empty_slot_ratio > p->full_ratio)) {
    t = 4;
    decide = 1;
  } else if (p->perf_enable && perf > 0.0 && perf_baseline > 0.0 &&
             perf < p->perf_degrad * perf_baseline) {
    t = 5;
    decide = 1;
  }
  if (trigger) *trigger = t;
  return decide;
}

// ----------------------------------------------------------------------------------
static void free_bins(pic_bins* b) {
  if (!b) return;
  int32_t* bufs[] = {b->kb.off, b->kb.len, b->kb.out_flag, b->kb.ins_cnt, b->kb.tile_flag,
                     b->kb.mv_slot, b->kb.mv_old, b->kb.mv_new, b->bin_cell, b->sbin,
                     b->scratch.id, b->scan_tmp[0], b->scan_tmp[1], b->scan_tmp[2],
                     b->scan_tmp[3]};
  for (int32_t* p : bufs)
    if (p) (void)hipFree(p);
  if (b->dctr) (void)hipFree(b->dctr);
  if (b->kb.wscr) (void)hipFree(b->kb.wscr);
  void* sp[] = {b->scratch.x, b->scratch.y, b->scratch.z, b->scratch.ux, b->scratch.uy,
                b->scratch.uz, b->scratch.w};
  for (void* p : sp)
    if (p) (void)hipFree(p);
  if (b->hstats) (void)hipHostFree(b->hstats);
  for (hipEvent_t ev : b->stats_ev)
    if (ev) (void)hipEventDestroy(ev);
  delete b;
}

template <typename T>
static hipError_t dalloc(T** p, int64_t n) {
  return hipMalloc((void**)p, (size_t)std::max<int64_t>(n, 1) * sizeof(T));
}

extern "C" pic_status pic_bins_create(const pic_grid* grid, const int tile[3], double slack,
                                      int64_t nslots, int64_t max_movers, pic_bins** out) {
  pic_status st = validate_grid(grid);
  if (st != PIC_OK) return st;
  if (!tile || !out) return set_error(PIC_ERR_INVALID_ARG, "tile and out must not be NULL");
  if (!(slack >= 0.0) || slack > 16.0) return set_error(PIC_ERR_INVALID_ARG, "slack must be in [0, 16]");
  if (nslots < 0 || nslots >= (1ll << 31) - 64)
    return set_error(PIC_ERR_INVALID_ARG, "nslots must be in [0, 2^31 - 64)");
  int T[3], nt[3], n[3];
  int64_t nbins = 1, ntiles = 1;
  for (int d = 0; d < 3; ++d) {
    n[d] = d < grid->dim ? grid->n[d] : 1;
    T[d] = d < grid->dim ? tile[d] : 1;
    if (T[d] < 1) return set_error(PIC_ERR_INVALID_ARG, "tile extents must be positive");
    if (T[d] > n[d]) T[d] = n[d];
    nt[d] = (n[d] + T[d] - 1) / T[d];
    nbins *= n[d];
    ntiles *= nt[d];
  }
  if ((int64_t)T[0] * T[1] * T[2] > 8192)
    return set_error(PIC_ERR_INVALID_ARG, "a tile may hold at most 8192 cells");
  for (int d = 0; d < grid->dim; ++d)
    if (T[d] < 4 && T[d] != n[d])
      return set_error(PIC_ERR_INVALID_ARG, "tile extents must be at least 4 cells (or the grid)");
  if (nbins >= (1ll << 31) - 1) return set_error(PIC_ERR_INVALID_ARG, "too many cells");
  if (max_movers <= 0) max_movers = nslots / 8 + 4096;
  if (max_movers >= (1ll << 31)) max_movers = (1ll << 31) - 1;

  pic_bins* b = new pic_bins();
  b->grid = *grid;
  b->nslots = nslots;
  b->slack = slack;
  for (int d = 0; d < 3; ++d) {
    b->kb.T[d] = T[d];
    b->kb.nt[d] = nt[d];
  }
  b->kb.nbins = (int32_t)nbins;
  b->kb.ntiles = (int32_t)ntiles;
  b->kb.max_movers = (int32_t)max_movers;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  A(dalloc(&b->kb.off, nbins + 1));
  A(dalloc(&b->kb.len, nbins));
  A(dalloc(&b->kb.out_flag, nbins));
  A(dalloc(&b->kb.ins_cnt, nbins));
  A(dalloc(&b->kb.tile_flag, ntiles));
  A(dalloc(&b->kb.mv_slot, max_movers));
  A(dalloc(&b->kb.mv_old, max_movers));
  A(dalloc(&b->kb.mv_new, max_movers));
  A(dalloc(&b->bin_cell, nbins));
  A(dalloc(&b->sbin, nslots));
  A(dalloc(&b->dctr, 2));
  {
    int64_t wm = 1;
    for (int d = 0; d < grid->dim; ++d) wm *= T[d] + 4;
    b->kb.wmax = (int32_t)wm;
    A(dalloc(&b->kb.wscr, ntiles * 3 * wm));
  }
  A(dalloc(&b->scratch.x, nslots));
  A(dalloc(&b->scratch.y, nslots));
  A(dalloc(&b->scratch.z, nslots));
  A(dalloc(&b->scratch.ux, nslots));
  A(dalloc(&b->scratch.uy, nslots));
  A(dalloc(&b->scratch.uz, nslots));
  A(dalloc(&b->scratch.w, nslots));
  A(dalloc(&b->scratch.id, nslots));
  b->scratch.nslots = (int32_t)nslots;
  // scan levels over nbins + 1 entries, 2048 per block
  int64_t m = nbins + 1;
  b->scan_n[0] = m;
  int lv = 0;
  while (m > 2048 && lv < 4) {
    m = (m + 2047) / 2048;
    A(dalloc(&b->scan_tmp[lv], m));
    b->scan_n[lv + 1] = m;
    ++lv;
  }
  b->scan_levels = lv;
  {
    int dev = 0, lds = 0;
    A(hipGetDevice(&dev));
    A(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if (lds > 0) b->max_lds = (size_t)lds;
  }
  A(hipHostMalloc((void**)&b->hstats, sizeof(CtrBlock) * STATS_RING, hipHostMallocDefault));
  for (hipEvent_t& ev : b->stats_ev) A(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  if (e != hipSuccess) {
    free_bins(b);
    return check_hip(e, "pic_bins_create allocation");
  }
  b->kb.ctr = b->dctr->ctr;
  b->kb.err = &b->dctr->err;
  // bin -> cell table (host computed once)
  std::vector<int32_t> bc((size_t)nbins);
  for (int k = 0; k < n[2]; ++k)
    for (int j = 0; j < n[1]; ++j)
      for (int i = 0; i < n[0]; ++i)
        bc[(size_t)bin_of_cell(n, T, i, j, k)] = (i + n[0] * (j + n[1] * k));
  A(hipMemcpy(b->bin_cell, bc.data(), bc.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  A(hipMemset(b->kb.off, 0, (size_t)(nbins + 1) * sizeof(int32_t)));
  A(hipMemset(b->kb.len, 0, (size_t)nbins * sizeof(int32_t)));
  A(hipMemset(b->kb.out_flag, 0, (size_t)nbins * sizeof(int32_t)));
  A(hipMemset(b->kb.ins_cnt, 0, (size_t)nbins * sizeof(int32_t)));
  A(hipMemset(b->kb.tile_flag, 0, (size_t)ntiles * sizeof(int32_t)));
  A(hipMemset(b->dctr, 0, 2 * sizeof(CtrBlock)));
  memset(b->hstats, 0, sizeof(CtrBlock) * STATS_RING);
  A(hipDeviceSynchronize());
  if (e != hipSuccess) {
    free_bins(b);
    return check_hip(e, "pic_bins_create initialisation");
  }
  *out = b;
  return PIC_OK;
}

extern "C" pic_status pic_bins_destroy(pic_bins* bins) {
  if (!bins) return PIC_OK;
  (void)hipDeviceSynchronize();
  free_bins(bins);
  return PIC_OK;
}

extern "C" pic_status pic_bins_get_view(const pic_bins* b, pic_bins_view* out) {
  if (!b || !out) return set_error(PIC_ERR_INVALID_ARG, "NULL argument");
  out->nbins = b->kb.nbins;
  out->ntiles = b->kb.ntiles;
  for (int d = 0; d < 3; ++d) out->ntile[d] = b->kb.nt[d];
  out->off = b->kb.off;
  out->len = b->kb.len;
  out->bin_cell = b->bin_cell;
  return PIC_OK;
}

extern "C" pic_status pic_bins_copy_tables(const pic_bins* b, int32_t* off_host, int32_t* len_host,
                                           int32_t* cell_host, hipStream_t stream) {
  if (!b) return set_error(PIC_ERR_INVALID_ARG, "bins is NULL");
  HIP_TRY(hipStreamSynchronize(stream));
  const size_t nb = (size_t)b->kb.nbins;
  if (off_host) HIP_TRY(hipMemcpy(off_host, b->kb.off, (nb + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (len_host) HIP_TRY(hipMemcpy(len_host, b->kb.len, nb * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (cell_host) HIP_TRY(hipMemcpy(cell_host, b->bin_cell, nb * sizeof(int32_t), hipMemcpyDeviceToHost));
  return PIC_OK;
}

static double empty_ratio_of(const CtrBlock& c) {
  const double cap = (double)c.cap_used;
  return cap > 0 ? 1.0 - (double)c.ctr[CTR_NVALID] / cap : 0.0;
}

static pic_rebin_record* record_of(pic_bins* b, int64_t seq) {
  if (seq < b->history_base || seq >= b->history_base + (int64_t)b->history.size()) return nullptr;
  return &b->history[(size_t)(seq - b->history_base)];
}

// Read the statistics of every call up to `upto` (in call order), waiting for each copy to
// land, and fold them into the policy state: local rebuilds of calls after the last full
// sort add up; the empty-slot ratio is that of the newest such call (the full sort's own
// statistics included).
static pic_status consume_stats(pic_bins* b, int64_t upto) {
  upto = std::min(upto, b->seq_enqueued - 1);
  while (b->seq_consumed <= upto) {
    const int64_t j = b->seq_consumed;
    const int slot = (int)(j % STATS_RING);
    HIP_TRY(hipEventSynchronize(b->stats_ev[slot]));
    const CtrBlock& c = b->hstats[slot];
    if (j > b->last_full_seq) b->rebuilds_since_sort += c.ctr[CTR_NREB];
    if (j >= b->last_full_seq) b->known_empty_ratio = empty_ratio_of(c);
    if (pic_rebin_record* r = record_of(b, j)) {
      r->n_valid = c.ctr[CTR_NVALID];
      r->n_moved = c.ctr[CTR_NMOV_LAST];
      r->n_overflow = c.ctr[CTR_NOVF];
      r->n_mover_drop = c.ctr[CTR_NDROP];
      r->n_local_rebuilds = c.ctr[CTR_NREB];
      r->error_flags = c.err;
      r->empty_slot_ratio = empty_ratio_of(c);
      r->complete = 1;
    }
    b->seq_consumed = j + 1;
  }
  return PIC_OK;
}

extern "C" pic_status pic_bins_report_perf(pic_bins* b, double perf) {
  if (!b) return set_error(PIC_ERR_INVALID_ARG, "bins is NULL");
  b->perf_last = perf;
  if (b->perf_baseline_pending) {
    b->perf_baseline = perf;
    b->perf_baseline_pending = false;
  }
  return PIC_OK;
}

extern "C" pic_status pic_rebin(const pic_grid* grid, pic_particles* p, pic_bins* b, int mode,
                                const pic_sort_policy* policy, hipStream_t stream) {
  pic_status st = validate_grid(grid);
  if (st != PIC_OK) return st;
  if ((st = validate_particles(p, grid->dim)) != PIC_OK) return st;
  if (!b) return set_error(PIC_ERR_INVALID_ARG, "bins is NULL");
  if (!same_grid(*grid, b->grid)) return set_error(PIC_ERR_INVALID_ARG, "grid differs from the bins' grid");
  if (p->nslots != b->nslots) return set_error(PIC_ERR_INVALID_ARG, "nslots differs from the bins' nslots");
  if (mode != PIC_REBIN_FULL && mode != PIC_REBIN_INCREMENTAL && mode != PIC_REBIN_AUTO)
    return set_error(PIC_ERR_INVALID_ARG, "unknown rebin mode");
  if (mode != PIC_REBIN_FULL && !b->sorted_once)
    return set_error(PIC_ERR_INVALID_ARG, "the first rebin must be PIC_REBIN_FULL");
  {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(stream, &cs));
    if (cs != hipStreamCaptureStatusNone)
      return set_error(PIC_ERR_UNSUPPORTED, "pic_rebin cannot be captured into a graph");
  }
  KGrid G = make_kgrid(*grid);
  KPart P = make_kpart(*p);
  const int64_t seq = b->seq_enqueued;
  // statistics the decision may use (and ring slots about to be reused) come back first
  if ((st = consume_stats(b, seq - POLICY_LAG)) != PIC_OK) return st;
  pic_rebin_record rec{};
  rec.seq = seq;
  rec.trigger = -1;
  rec.steps_since_sort = b->steps_since_sort;
  rec.rebuilds_since_sort = b->rebuilds_since_sort;
  rec.known_empty_ratio = b->known_empty_ratio;
  int run = mode;
  if (mode == PIC_REBIN_AUTO) {
    int trig = 0;
    int dec = pic_policy_decide(policy, b->steps_since_sort, b->rebuilds_since_sort,
                                b->known_empty_ratio, b->perf_last, b->perf_baseline, &trig);
    b->last_decision = dec;
    rec.trigger = trig;
    run = dec ? PIC_REBIN_FULL : PIC_REBIN_INCREMENTAL;
  }
  if (run == PIC_REBIN_FULL) {
    rebin_full(b, G, P, stream);
    b->sorted_once = true;
    b->steps_since_sort = 0;
    b->rebuilds_since_sort = 0;
    b->last_full_seq = seq;
    b->known_empty_ratio = -1.0;
    b->n_global_sorts++;
    b->perf_baseline_pending = true;
  } else {
    rebin_incremental(b, G, P, stream);
    b->steps_since_sort++;
  }
  rec.mode = run;
  b->movers_fresh = false;
  b->last_mode = run;
  if (b->history.size() >= HISTORY_MAX) {
    b->history.pop_front();
    b->history_base++;
  }
  if (b->history.empty()) b->history_base = seq;
  b->history.push_back(rec);
  // statistics: device counters (snapshot) -> this call's pinned ring slot, read later in
  // call order; the per-rebin counters restart from zero in the same kernel
  const int slot = (int)(seq % STATS_RING);
  rebin_finish(b, stream);
  HIP_TRY(hipMemcpyAsync(&b->hstats[slot], b->dctr + 1, sizeof(CtrBlock), hipMemcpyDeviceToHost,
                         stream));
  HIP_TRY(hipEventRecord(b->stats_ev[slot], stream));
  b->seq_enqueued = seq + 1;
  return check_hip(hipGetLastError(), "pic_rebin launch");
}

extern "C" pic_status pic_rebin_stats_read(pic_bins* b, hipStream_t stream, pic_rebin_stats* out) {
  if (!b || !out) return set_error(PIC_ERR_INVALID_ARG, "NULL argument");
  HIP_TRY(hipStreamSynchronize(stream));
  pic_status st = consume_stats(b, b->seq_enqueued - 1);
  if (st != PIC_OK) return st;
  const CtrBlock& c = b->hstats[(int)((b->seq_enqueued + STATS_RING - 1) % STATS_RING)];
  out->n_valid = c.ctr[CTR_NVALID];
  out->n_moved = c.ctr[CTR_NMOV_LAST];
  out->n_overflow = c.ctr[CTR_NOVF];
  out->n_mover_drop = c.ctr[CTR_NDROP];
  out->n_local_rebuilds = c.ctr[CTR_NREB];
  out->n_global_sorts = b->n_global_sorts;
  double cap = (double)c.cap_used;
  out->empty_slot_ratio = cap > 0 ? 1.0 - (double)c.ctr[CTR_NVALID] / cap : 0.0;
  out->global_sort_recommended = pic_policy_decide(
      nullptr, b->steps_since_sort, b->rebuilds_since_sort, out->empty_slot_ratio, b->perf_last,
      b->perf_baseline, nullptr);
  out->last_mode = b->last_mode;
  out->error_flags = c.err;
  return PIC_OK;
}

extern "C" pic_status pic_rebin_history(pic_bins* b, hipStream_t stream, int64_t first,
                                        int32_t max, pic_rebin_record* out, int32_t* count) {
  if (!b || !count || (max > 0 && !out)) return set_error(PIC_ERR_INVALID_ARG, "NULL argument");
  if (first < 0 || max < 0) return set_error(PIC_ERR_INVALID_ARG, "first and max must be >= 0");
  *count = 0;
  HIP_TRY(hipStreamSynchronize(stream));
  pic_status st = consume_stats(b, b->seq_enqueued - 1);
  if (st != PIC_OK) return st;
  int32_t n = 0;
  for (int64_t q = std::max(first, b->history_base); n < max; ++q) {
    const pic_rebin_record* r = record_of(b, q);
    if (!r) break;
    out[n++] = *r;
  }
  *count = n;
  return PIC_OK;
}

// Argument checks of pic_deposit (and its no-allocation variant).
pic_status deposit_check_args(const pic_grid* grid, const pic_particles* p, const pic_bins* b,
                              const float* Jx, const float* Jy, const float* Jz, int path,
                              unsigned flags) {
  pic_status st = validate_grid(grid);
  if (st != PIC_OK) return st;
  if ((st = validate_particles(p, grid->dim)) != PIC_OK) return st;
  if (!Jx || !Jy || !Jz) return set_error(PIC_ERR_INVALID_ARG, "J pointers must not be NULL");
  if (flags & ~(unsigned)(PIC_F_ACCUMULATE | PIC_F_EMIT_MOVERS | PIC_F_DRIFT |
                          PIC_F_MIDPOINT))
    return set_error(PIC_ERR_INVALID_ARG, "unknown flag bits");
  if (path < PIC_PATH_AUTO || path > PIC_PATH_UNSORTED)
    return set_error(PIC_ERR_INVALID_ARG, "unknown deposition path");
  if ((flags & PIC_F_MIDPOINT) && path != PIC_PATH_AUTO && path != PIC_PATH_CELL_VALU &&
      path != PIC_PATH_UNSORTED)
    return set_error(PIC_ERR_UNSUPPORTED, "PIC_F_MIDPOINT runs on the per-cell and unsorted paths");
  if (path != PIC_PATH_UNSORTED) {
    if (!b) return set_error(PIC_ERR_INVALID_ARG, "bins required for this path");
    if (!same_grid(*grid, b->grid)) return set_error(PIC_ERR_INVALID_ARG, "grid differs from the bins' grid");
    if (p->nslots != b->nslots) return set_error(PIC_ERR_INVALID_ARG, "nslots differs from the bins' nslots");
    if (!b->sorted_once) return set_error(PIC_ERR_INVALID_ARG, "bins are empty: run pic_rebin(PIC_REBIN_FULL) first");
  } else if (flags & PIC_F_EMIT_MOVERS) {
    return set_error(PIC_ERR_INVALID_ARG, "PIC_F_EMIT_MOVERS needs bins");
  }
  if ((flags & (PIC_F_DRIFT | PIC_F_MIDPOINT)) && !std::isfinite(grid->dt))
    return set_error(PIC_ERR_INVALID_ARG, "dt must be finite");
  return PIC_OK;
}

// Enqueue a checked deposition; the tile windows go to `wscr` (the bins' own when NULL).
pic_status deposit_enqueue(const pic_grid* grid, pic_particles* p, pic_bins* b, float* Jx,
                           float* Jy, float* Jz, int path, unsigned flags, float* wscr,
                           hipStream_t stream) {
  KGrid G = make_kgrid(*grid);
  KPart P = make_kpart(*p);
  pic_bins* bb = path == PIC_PATH_UNSORTED ? nullptr : b;
  float* own = bb ? bb->kb.wscr : nullptr;
  if (bb && wscr) bb->kb.wscr = wscr;      // kernels take the bins by value at launch
  const bool ok = deposit_launch(G, P, bb, Jx, Jy, Jz, path, flags, grid->dt, stream);
  if (bb) bb->kb.wscr = own;
  if (!ok) return set_error(PIC_ERR_UNSUPPORTED, "deposition path not available for this grid");
  if (b) {
    if (flags & PIC_F_EMIT_MOVERS) b->movers_fresh = true;
    else if (flags & PIC_F_DRIFT) b->movers_fresh = false;
  }
  return check_hip(hipGetLastError(), "pic_deposit launch");
}

extern "C" pic_status pic_deposit(const pic_grid* grid, pic_particles* p, pic_bins* b, float* Jx,
                                  float* Jy, float* Jz, int path, unsigned flags,
                                  hipStream_t stream) {
  pic_status st = deposit_check_args(grid, p, b, Jx, Jy, Jz, path, flags);
  if (st != PIC_OK) return st;
  return deposit_enqueue(grid, p, b, Jx, Jy, Jz, path, flags, nullptr, stream);
}

extern "C" pic_status pic_deposit_rho(const pic_grid* grid, const pic_particles* p, pic_bins* b,
                                      float* rho, unsigned flags, hipStream_t stream) {
  pic_status st = validate_grid(grid);
  if (st != PIC_OK) return st;
  if ((st = validate_particles(p, grid->dim)) != PIC_OK) return st;
  if (!rho) return set_error(PIC_ERR_INVALID_ARG, "rho must not be NULL");
  if (flags & ~(unsigned)PIC_F_ACCUMULATE)
    return set_error(PIC_ERR_INVALID_ARG, "pic_deposit_rho takes PIC_F_ACCUMULATE only");
  if (!b) return set_error(PIC_ERR_INVALID_ARG, "bins required");
  if (!same_grid(*grid, b->grid)) return set_error(PIC_ERR_INVALID_ARG, "grid differs from the bins' grid");
  if (p->nslots != b->nslots) return set_error(PIC_ERR_INVALID_ARG, "nslots differs from the bins' nslots");
  if (!b->sorted_once) return set_error(PIC_ERR_INVALID_ARG, "bins are empty: run pic_rebin(PIC_REBIN_FULL) first");
  KGrid G = make_kgrid(*grid);
  KPart P = make_kpart(*p);
  if (!(flags & PIC_F_ACCUMULATE)) launch_fill_f32(rho, (int64_t)G.N[0] * G.N[1] * G.N[2], 0.0f, stream);
  if (!deposit_rho_cell_launch(G, P, b, rho, stream))
    return set_error(PIC_ERR_UNSUPPORTED, "tile window too large for LDS");
  halo_rho_launch(G, b, rho, stream);
  return check_hip(hipGetLastError(), "pic_deposit_rho launch");
}

extern "C" pic_status pic_deposit_backward(const pic_grid* grid, const pic_particles* p,
                                           const pic_bins* b, const float* Gx, const float* Gy,
                                           const float* Gz, float* dx, float* dy, float* dz,
                                           float* dux, float* duy, float* duz, float* dw,
                                           unsigned flags, hipStream_t stream) {
  pic_status st = validate_grid(grid);
  if (st != PIC_OK) return st;
  if ((st = validate_particles(p, grid->dim)) != PIC_OK) return st;
  if (!Gx || !Gy || !Gz || !dx || !dy || (grid->dim == 3 && !dz) || !dux || !duy || !duz)
    return set_error(PIC_ERR_INVALID_ARG, "gradient pointers must not be NULL");
  if (flags != 0) return set_error(PIC_ERR_INVALID_ARG, "pic_deposit_backward takes no flags");
  if (b && !same_grid(*grid, b->grid)) return set_error(PIC_ERR_INVALID_ARG, "grid differs from the bins' grid");
  KGrid G = make_kgrid(*grid);
  KPart P = make_kpart(*p);
  backward_launch(G, P, b, Gx, Gy, Gz, dx, dy, grid->dim == 3 ? dz : nullptr, dux, duy, duz, dw,
                  stream);
  return check_hip(hipGetLastError(), "pic_deposit_backward launch");
}

extern "C" pic_status pic_drift(const pic_grid* grid, pic_particles* p, double dt, hipStream_t stream) {
  pic_status st = validate_grid(grid);
  if (st != PIC_OK) return st;
  if ((st = validate_particles(p, grid->dim)) != PIC_OK) return st;
  if (!std::isfinite(dt)) return set_error(PIC_ERR_INVALID_ARG, "dt must be finite");
  drift_launch(make_kgrid(*grid), make_kpart(*p), dt, stream);
  return check_hip(hipGetLastError(), "pic_drift launch");
}

extern "C" pic_status pic_check(pic_bins* b, hipStream_t stream) {
  HIP_TRY(hipStreamSynchronize(stream));
  if (!b) return PIC_OK;
  uint32_t err = 0;
  HIP_TRY(hipMemcpy(&err, b->kb.err, sizeof(uint32_t), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(b->kb.err, 0, sizeof(uint32_t)));
  if (err & PIC_EF_NONFINITE) return set_error(PIC_ERR_INVALID_PARTICLE, "non-finite particle position");
  if (err & PIC_EF_MOVE)
    return set_error(PIC_ERR_INVALID_PARTICLE, "a particle moved a cell or more in one step");
  if (err & (PIC_EF_DOMAIN | PIC_EF_STENCIL)) return set_error(PIC_ERR_OUT_OF_DOMAIN, "particle outside the domain");
  if (err & PIC_EF_CAPACITY) return set_error(PIC_ERR_CAPACITY, "particle arrays too small for the bins");
  return PIC_OK;
}
