// pic_deposit_noalloc: pic_deposit with its tile-window scratch (the per-tile stencil
// windows the deposition kernel writes and the window-sum kernel reads back) in a fixed
// device array of this library instead of the bins' own allocation. It allocates nothing
// and never calls the HIP allocator; its limit is the size of that array.
#include <mutex>

#include "pic_host.h"

// The window scratch of every pic_deposit_noalloc call on one GPU. Each GPU the library
// runs on holds its own copy until the process ends. In host code `scratch` only names
// the symbol: its device address comes from hipGetSymbolAddress (scratch_ptr below).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES];
static std::once_flag g_scratch_once[NOALLOC_MAX_DEVICES];
static hipError_t g_scratch_err[NOALLOC_MAX_DEVICES];

// Device address of the current device's `scratch` (looked up once per device, with that
// device current).
static pic_status scratch_ptr(void** out) {
  int dev = 0;
  pic_status st = check_hip(hipGetDevice(&dev), "pic_deposit_noalloc: hipGetDevice");
  if (st != PIC_OK) return st;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return set_error(PIC_ERR_UNSUPPORTED, "pic_deposit_noalloc: device ordinal above 63");
  std::call_once(g_scratch_once[dev], [dev]() {
    void* p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? p : nullptr;
  });
  if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev])
    return check_hip(g_scratch_err[dev] != hipSuccess ? g_scratch_err[dev] : hipErrorInvalidSymbol,
                     "pic_deposit_noalloc: hipGetSymbolAddress(scratch)");
  *out = g_scratch_ptr[dev];
  return PIC_OK;
}

extern "C" pic_status pic_deposit_noalloc(const pic_grid* grid, pic_particles* p, pic_bins* b,
                                          float* Jx, float* Jy, float* Jz, int path,
                                          unsigned flags, hipStream_t stream) {
  pic_status st = deposit_check_args(grid, p, b, Jx, Jy, Jz, path, flags);
  if (st != PIC_OK) return st;
  float* wscr = nullptr;
  if (path != PIC_PATH_UNSORTED) {
    const size_t need = (size_t)b->kb.ntiles * 3 * (size_t)b->kb.wmax * sizeof(float);
    if (need > NOALLOC_SCRATCH_BYTES)
      return set_error(PIC_ERR_INVALID_ARG,
                       "pic_deposit_noalloc: the tile windows need " + std::to_string(need) +
                           " bytes of scratch, above the fixed " +
                           std::to_string(NOALLOC_SCRATCH_BYTES) + " (use pic_deposit)");
    void* sp = nullptr;
    if ((st = scratch_ptr(&sp)) != PIC_OK) return st;
    wscr = (float*)sp;
  }
  return deposit_enqueue(grid, p, b, Jx, Jy, Jz, path, flags, wscr, stream);
}
