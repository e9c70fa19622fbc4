// Batched deposition over many independent patches (persistent launch).
#include "deposit_common.h"

struct pic_plan {
  int npatch;
};

extern "C" pic_status pic_plan_create(const pic_grid* grids, int npatch, pic_bins* const* bins,
                                      const char* tune_cache_json, pic_plan** out) {
  (void)grids; (void)npatch; (void)bins; (void)tune_cache_json; (void)out;
  return set_error(PIC_ERR_UNSUPPORTED, "batched plans are not built yet");
}

extern "C" pic_status pic_plan_destroy(pic_plan* plan) {
  delete plan;
  return PIC_OK;
}

extern "C" pic_status pic_deposit_batched(pic_plan* plan, const pic_particles* particles,
                                          float* const* J3, int path, unsigned flags,
                                          hipStream_t stream) {
  (void)plan; (void)particles; (void)J3; (void)path; (void)flags; (void)stream;
  return set_error(PIC_ERR_UNSUPPORTED, "batched plans are not built yet");
}
