// Host-side state of libpic objects and the launchers each kernel file provides.
#pragma once

#include <deque>
#include <string>

#include "pic_internal.h"

// Device counter block: CTR_COUNT int32 counters, the error word, the slot count used by
// the bins and two 64-bit accumulators, copied to pinned host memory after every rebin.
struct CtrBlock {
  int32_t ctr[CTR_COUNT];
  uint32_t err;
  int32_t cap_used;           // off[nbins]: slots inside bins
  unsigned long long desired; // full sort: extra slots wanted
  unsigned long long pad;
};

// Statistics of rebin calls come back through a ring of pinned counter blocks, one per
// call. The policy of call s reads the statistics of every call up to s - POLICY_LAG,
// waiting for them if they have not landed, so its decisions do not depend on how far
// the host runs ahead of the device (it runs at most POLICY_LAG rebins ahead).
constexpr int STATS_RING = 8;
constexpr int POLICY_LAG = 2;
static_assert(STATS_RING > POLICY_LAG, "a ring slot is reused only after it was consumed");
constexpr size_t HISTORY_MAX = 1u << 16;   // rebin records kept per bins object

struct pic_bins {
  pic_grid grid;
  KBins kb;
  int64_t nslots;
  double slack;
  size_t max_lds = 65536;           // LDS bytes a workgroup may use on this device
  // device buffers owned by the bins
  int32_t* bin_cell = nullptr;
  int32_t* sbin = nullptr;          // full sort: bin of every slot
  CtrBlock* dctr = nullptr;         // [0] live counters, [1] snapshot at the end of a rebin
  KPart scratch{};                  // full sort / rebuild staging, nslots slots
  // scan temporaries (levels of block sums)
  int32_t* scan_tmp[4] = {nullptr, nullptr, nullptr, nullptr};
  int64_t scan_n[5] = {0, 0, 0, 0, 0};
  int scan_levels = 0;
  // host-side state
  bool movers_fresh = false;
  bool sorted_once = false;
  CtrBlock* hstats = nullptr;       // pinned ring, STATS_RING blocks
  hipEvent_t stats_ev[STATS_RING] = {};
  int64_t seq_enqueued = 0;         // rebin calls whose statistics copy was enqueued
  int64_t seq_consumed = 0;         // calls whose statistics the host has read
  int last_mode = -1;
  // policy state (Sec. 4.4), as known to the host after consuming statistics
  int steps_since_sort = 0;
  int rebuilds_since_sort = 0;
  int n_global_sorts = 0;
  int64_t last_full_seq = -1;       // call number of the last full sort
  double known_empty_ratio = -1.0;  // of the newest consumed call since that sort; -1 unknown
  int last_decision = 0;
  double perf_baseline = -1.0;
  double perf_last = -1.0;
  bool perf_baseline_pending = true;
  // per-call records (decision inputs, then the statistics once consumed)
  std::deque<pic_rebin_record> history;
  int64_t history_base = 0;         // seq of history.front()
};

// Zero fill of int32 device memory (rebin.hip).
__global__ void k_zero_i32(int32_t* p, int64_t n);

// Launchers (implemented in rebin.hip / deposit.hip / backward.hip).
KGrid make_kgrid(const pic_grid& g);
KPart make_kpart(const pic_particles& p);
void rebin_full(pic_bins* b, const KGrid& G, const KPart& P, hipStream_t s);
void rebin_incremental(pic_bins* b, const KGrid& G, const KPart& P, hipStream_t s);
void rebin_finish(pic_bins* b, hipStream_t s);
bool deposit_launch(const KGrid& G, const KPart& P, pic_bins* b, float* J0, float* J1,
                    float* J2, int path, unsigned flags, double dt, hipStream_t s);
void drift_launch(const KGrid& G, const KPart& P, double dt, hipStream_t s);
void backward_launch(const KGrid& G, const KPart& P, const pic_bins* b, const float* G0,
                     const float* G1, const float* G2, float* dx, float* dy, float* dz,
                     float* dux, float* duy, float* duz, float* dw, hipStream_t s);
void scan_exclusive_i32(pic_bins* b, int32_t* data, int64_t n, hipStream_t s);
void reset_movers(pic_bins* b, hipStream_t s);

// Argument checks shared by the entry points (api.hip).
pic_status validate_grid(const pic_grid* g);
pic_status validate_particles(const pic_particles* p, int dim);
bool same_grid(const pic_grid& a, const pic_grid& b);

// pic_deposit's argument checks and launch, shared with its no-allocation variant (api.hip).
pic_status deposit_check_args(const pic_grid* grid, const pic_particles* p, const pic_bins* b,
                              const float* Jx, const float* Jy, const float* Jz, int path,
                              unsigned flags);
pic_status deposit_enqueue(const pic_grid* grid, pic_particles* p, pic_bins* b, float* Jx,
                           float* Jy, float* Jz, int path, unsigned flags, float* wscr,
                           hipStream_t stream);

// Error reporting (api.hip).
pic_status set_error(pic_status st, const std::string& msg);
pic_status check_hip(hipError_t e, const char* what);
