// Batched deposition over many independent 3D patches: one persistent launch.
//
// The paper decomposes each rank's domain into tiles (Sec. 4.1) and processes them one
// after another; here many patches of uneven size, density and shape order share one
// device-wide work list of (patch, tile) items. A plan fixes the patches, their bins and
// the work list (longest items first, by particles per tile x stencil volume); every call
// then enqueues three kernels (zero J / reset counters, the persistent per-cell
// deposition pulling items from a device counter, the tile-window sum into J, one
// workgroup per item), with no
// allocation, no host synchronisation and no memset node, so it can be captured into a
// HIP graph.
#include <algorithm>
#include <cstring>
#include <fstream>
#include <sstream>
#include <vector>

#include "deposit_common.h"

struct pic_plan {
  int npatch = 0;
  std::vector<pic_grid> grids;
  std::vector<pic_bins*> bins;
  BatchPatch* d_pd = nullptr;        // device descriptors
  BatchPatch* h_pd = nullptr;        // pinned staging of the descriptors
  std::vector<BatchPatch> last;      // descriptors last uploaded
  bool uploaded = false;
  hipEvent_t upload_ev = nullptr;
  int2* d_items = nullptr;           // every patch's tiles
  int nitems = 0;
  int2* d_items_vec = nullptr;       // tiles of the patches AUTO runs on the per-cell path
  int nitems_vec = 0;
  int2* d_rows = nullptr;            // window sum: (patch, first tile of a row of tiles)
  int nrows = 0;
  int2* d_rows_vec = nullptr;        // the same for the per-cell patches
  int nrows_vec = 0;
  std::vector<int> patch_path;       // PIC_PATH_AUTO's choice per patch (at plan creation)
  int* d_queue = nullptr;
  size_t smem = 0;
  size_t halo_smem = 0;
  int blocks = 0;
  int blocks_per_cu = 0;
  int64_t max_nodes = 0;
};

// The one setting the plan reads from the tuning cache: "blocks_per_cu": <int>
// (persistent workgroups per compute unit). Tile shapes in the cache are applied when the
// bins are made, before the plan.
static int read_blocks_per_cu(const char* path) {
  if (!path) return 0;
  std::ifstream f(path);
  if (!f) return -1;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  const std::string key = "\"blocks_per_cu\"";
  size_t k = t.find(key);
  if (k == std::string::npos) return 0;
  k = t.find(':', k + key.size());
  if (k == std::string::npos) return -1;
  return std::atoi(t.c_str() + k + 1);
}

static void plan_free(pic_plan* p) {
  if (!p) return;
  if (p->d_pd) (void)hipFree(p->d_pd);
  if (p->h_pd) (void)hipHostFree(p->h_pd);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_items_vec) (void)hipFree(p->d_items_vec);
  if (p->d_rows) (void)hipFree(p->d_rows);
  if (p->d_rows_vec) (void)hipFree(p->d_rows_vec);
  if (p->d_queue) (void)hipFree(p->d_queue);
  if (p->upload_ev) (void)hipEventDestroy(p->upload_ev);
  delete p;
}

extern "C" pic_status pic_plan_create(const pic_grid* grids, int npatch, pic_bins* const* bins,
                                      const char* tune_cache_json, pic_plan** out) {
  if (!out) return set_error(PIC_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!grids || !bins || npatch < 1 || npatch > 65535)
    return set_error(PIC_ERR_INVALID_ARG, "need 1..65535 patches with grids and bins");
  const int bpc = read_blocks_per_cu(tune_cache_json);
  if (bpc < 0) return set_error(PIC_ERR_INVALID_ARG, "tuning cache unreadable or malformed");
  pic_plan* p = new pic_plan();
  p->npatch = npatch;
  struct Item { int patch, tile; double cost; };
  std::vector<Item> items;
  size_t max_lds = 0;
  for (int k = 0; k < npatch; ++k) {
    pic_status st = validate_grid(&grids[k]);
    if (st != PIC_OK) { plan_free(p); return st; }
    if (grids[k].dim != 3) {
      plan_free(p);
      return set_error(PIC_ERR_UNSUPPORTED, "batched plans take 3D patches");
    }
    if (!bins[k] || !same_grid(grids[k], bins[k]->grid)) {
      plan_free(p);
      return set_error(PIC_ERR_INVALID_ARG, "each patch needs bins made for its grid");
    }
    const KBins& kb = bins[k]->kb;
    const size_t sm = cell_smem_bytes(grids[k].order, 3, kb);
    if (sm > bins[k]->max_lds) {
      plan_free(p);
      return set_error(PIC_ERR_UNSUPPORTED, "tile too large for LDS in a batched launch");
    }
    p->smem = std::max(p->smem, sm);
    p->halo_smem = std::max(p->halo_smem, halo_smem_bytes(kb));
    max_lds = bins[k]->max_lds;
    p->grids.push_back(grids[k]);
    p->bins.push_back(bins[k]);
    const KGrid G = make_kgrid(grids[k]);
    p->max_nodes = std::max<int64_t>(p->max_nodes, (int64_t)G.N[0] * G.N[1] * G.N[2]);
    const double per_tile = (double)bins[k]->nslots / (double)kb.ntiles;
    const double o1 = grids[k].order + 1.0;
    for (int t = 0; t < kb.ntiles; ++t) items.push_back({k, t, per_tile * (o1 * o1 * (o1 + 1.0))});
    const int ch = choose_path(G, bins[k]);
    p->patch_path.push_back(ch == PIC_PATH_MFMA_BF16 || ch == PIC_PATH_MFMA_FP16 ? ch
                                                                             : PIC_PATH_CELL_VALU);
  }
  (void)max_lds;
  std::stable_sort(items.begin(), items.end(),
                   [](const Item& a, const Item& b) { return a.cost > b.cost; });
  p->nitems = (int)items.size();
  std::vector<int2> h_items(items.size()), h_vec;
  for (size_t i = 0; i < items.size(); ++i) {
    h_items[i] = make_int2(items[i].patch, items[i].tile);
    if (p->patch_path[items[i].patch] == PIC_PATH_CELL_VALU) h_vec.push_back(h_items[i]);
  }
  p->nitems_vec = (int)h_vec.size();
  // window-sum items: rows of up to halo_row_tiles() tiles along x
  std::vector<int2> h_rows, h_rows_vec;
  const int gxr = halo_row_tiles();
  for (int k = 0; k < npatch; ++k) {
    const KBins& kb = bins[k]->kb;
    for (int r = 0; r < kb.nt[1] * kb.nt[2]; ++r)
      for (int x = 0; x < kb.nt[0]; x += gxr) {
        h_rows.push_back(make_int2(k, x + kb.nt[0] * r));
        if (p->patch_path[k] == PIC_PATH_CELL_VALU) h_rows_vec.push_back(h_rows.back());
      }
  }
  p->nrows = (int)h_rows.size();
  p->nrows_vec = (int)h_rows_vec.size();
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipMalloc(&p->d_pd, sizeof(BatchPatch) * npatch);
  if (e == hipSuccess) e = hipHostMalloc(&p->h_pd, sizeof(BatchPatch) * npatch, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc(&p->d_items, sizeof(int2) * h_items.size());
  if (e == hipSuccess) e = hipMalloc(&p->d_items_vec, sizeof(int2) * std::max<size_t>(h_vec.size(), 1));
  if (e == hipSuccess && !h_vec.empty())
    e = hipMemcpy(p->d_items_vec, h_vec.data(), sizeof(int2) * h_vec.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&p->d_rows, sizeof(int2) * std::max<size_t>(h_rows.size(), 1));
  if (e == hipSuccess) e = hipMalloc(&p->d_rows_vec, sizeof(int2) * std::max<size_t>(h_rows_vec.size(), 1));
  if (e == hipSuccess && !h_rows.empty())
    e = hipMemcpy(p->d_rows, h_rows.data(), sizeof(int2) * h_rows.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !h_rows_vec.empty())
    e = hipMemcpy(p->d_rows_vec, h_rows_vec.data(), sizeof(int2) * h_rows_vec.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&p->d_queue, sizeof(int) * 4);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->upload_ev, hipEventDisableTiming);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_items, h_items.data(), sizeof(int2) * h_items.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    plan_free(p);
    return check_hip(e, "pic_plan_create");
  }
  const int occ = batched_blocks_per_cu(p->smem);
  p->blocks_per_cu = bpc > 0 ? std::min(bpc, occ) : occ;
  p->blocks = std::max(1, std::min(p->nitems, p->blocks_per_cu * std::max(ncu, 1)));
  *out = p;
  return PIC_OK;
}

extern "C" pic_status pic_plan_destroy(pic_plan* plan) {
  if (plan) (void)hipDeviceSynchronize();
  plan_free(plan);
  return PIC_OK;
}

extern "C" pic_status pic_deposit_batched(pic_plan* plan, const pic_particles* particles,
                                          float* const* J3, int path, unsigned flags,
                                          hipStream_t stream) {
  if (!plan || !particles || !J3) return set_error(PIC_ERR_INVALID_ARG, "NULL argument");
  if (path != PIC_PATH_AUTO && path != PIC_PATH_CELL_VALU)
    return set_error(PIC_ERR_UNSUPPORTED, "batched launches take PIC_PATH_AUTO or PIC_PATH_CELL_VALU");
  if (flags & ~(unsigned)(PIC_F_ACCUMULATE | PIC_F_EMIT_MOVERS | PIC_F_DRIFT |
                          PIC_F_MIDPOINT))
    return set_error(PIC_ERR_INVALID_ARG, "unknown flag bits");
  std::vector<BatchPatch> pd(plan->npatch);
  for (int k = 0; k < plan->npatch; ++k) {
    const pic_grid& g = plan->grids[k];
    pic_bins* b = plan->bins[k];
    pic_status st = validate_particles(&particles[k], 3);
    if (st != PIC_OK) return st;
    if (particles[k].nslots != b->nslots)
      return set_error(PIC_ERR_INVALID_ARG, "nslots differs from the patch's bins");
    if (!b->sorted_once)
      return set_error(PIC_ERR_INVALID_ARG, "bins are empty: run pic_rebin(PIC_REBIN_FULL) first");
    if (!J3[3 * k] || !J3[3 * k + 1] || !J3[3 * k + 2])
      return set_error(PIC_ERR_INVALID_ARG, "J pointers must not be NULL");
    if ((flags & (PIC_F_DRIFT | PIC_F_MIDPOINT)) && !std::isfinite(g.dt))
      return set_error(PIC_ERR_INVALID_ARG, "dt must be finite");
    std::memset(&pd[k], 0, sizeof(BatchPatch));
    pd[k].G = make_kgrid(g);
    pd[k].B = b->kb;
    pd[k].P = make_kpart(particles[k]);
    for (int c = 0; c < 3; ++c) pd[k].J[c] = J3[3 * k + c];
    pd[k].dt = g.dt;
  }
  const bool same = plan->uploaded &&
                    std::memcmp(pd.data(), plan->last.data(), sizeof(BatchPatch) * pd.size()) == 0;
  if (!same) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cs);
    if (e != hipSuccess) return check_hip(e, "pic_deposit_batched");
    if (cs != hipStreamCaptureStatusNone)
      return set_error(PIC_ERR_INVALID_ARG,
                       "new particle or J pointers during graph capture: call once outside "
                       "the capture with the same pointers first");
    if (plan->uploaded && (e = hipEventSynchronize(plan->upload_ev)) != hipSuccess)
      return check_hip(e, "pic_deposit_batched");
    std::memcpy(plan->h_pd, pd.data(), sizeof(BatchPatch) * pd.size());
    e = hipMemcpyAsync(plan->d_pd, plan->h_pd, sizeof(BatchPatch) * pd.size(),
                       hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(plan->upload_ev, stream);
    if (e != hipSuccess) return check_hip(e, "pic_deposit_batched upload");
    plan->last = pd;
    plan->uploaded = true;
  }
  // AUTO follows the plan's per-patch choice (the matrix paths have no midpoint deposition:
  // with PIC_F_MIDPOINT every patch runs on the per-cell path)
  const bool split = path == PIC_PATH_AUTO && !(flags & PIC_F_MIDPOINT) &&
                     plan->nitems_vec < plan->nitems;
  const int2* items = split ? plan->d_items_vec : plan->d_items;
  const int nitems = split ? plan->nitems_vec : plan->nitems;
  batched_prologue_launch(plan->d_pd, plan->npatch, plan->max_nodes, plan->d_queue, flags, stream);
  if (nitems > 0) {
    batched_cell_launch(plan->d_pd, items, nitems, plan->d_queue, plan->blocks, plan->smem, flags,
                        stream);
    batched_halo_tile_launch(plan->d_pd, split ? plan->d_rows_vec : plan->d_rows,
                             split ? plan->nrows_vec : plan->nrows, plan->halo_smem, stream);
  }
  if (split) {
    // patches on a matrix path: their own launches, J already cleared by the prologue
    for (int k = 0; k < plan->npatch; ++k) {
      if (plan->patch_path[k] == PIC_PATH_CELL_VALU) continue;
      if (!deposit_launch(pd[k].G, pd[k].P, plan->bins[k], J3[3 * k], J3[3 * k + 1],
                          J3[3 * k + 2], plan->patch_path[k], flags | PIC_F_ACCUMULATE,
                          plan->grids[k].dt, stream))
        return set_error(PIC_ERR_UNSUPPORTED, "matrix path not available for a patch");
    }
  }
  for (int k = 0; k < plan->npatch; ++k) {
    if (flags & PIC_F_EMIT_MOVERS) plan->bins[k]->movers_fresh = true;
    else if (flags & PIC_F_DRIFT) plan->bins[k]->movers_fresh = false;
  }
  return check_hip(hipGetLastError(), "pic_deposit_batched launch");
}

extern "C" pic_status pic_plan_patch_path(const pic_plan* plan, int patch, int* path) {
  if (!plan || !path) return set_error(PIC_ERR_INVALID_ARG, "NULL argument");
  if (patch < 0 || patch >= plan->npatch) return set_error(PIC_ERR_INVALID_ARG, "no such patch");
  *path = plan->patch_path[patch];
  return PIC_OK;
}

extern "C" pic_status pic_plan_info(const pic_plan* plan, int* nitems, int* blocks,
                                    int* blocks_per_cu, int64_t* lds_bytes) {
  if (!plan) return set_error(PIC_ERR_INVALID_ARG, "plan is NULL");
  if (nitems) *nitems = plan->nitems;
  if (blocks) *blocks = plan->blocks;
  if (blocks_per_cu) *blocks_per_cu = plan->blocks_per_cu;
  if (lds_bytes) *lds_bytes = (int64_t)plan->smem;
  return PIC_OK;
}
