// Split-precision MFMA deposition (placeholder until the kernel lands).
#include "deposit_common.h"

bool deposit_mfma_launch(const KGrid& G, const KPart& P, pic_bins* b, float* J0, float* J1,
                         float* J2, int path, unsigned flags, double dt, hipStream_t s) {
  (void)G; (void)P; (void)b; (void)J0; (void)J1; (void)J2; (void)path; (void)flags; (void)dt; (void)s;
  return false;
}
