// Tile machinery shared by the bin-based deposition kernels: the LDS window a tile
// accumulates into, slot -> bin lookup, and the window -> J reduction.
#pragma once

#include <algorithm>

#include "particle.h"
#include "pic_host.h"

// Stencil window of a tile: all nodes any particle of the tile's cells can reach.
// Along each used dimension it starts LO nodes before the tile's first cell and spans
// extent + R nodes (order 1: [-1, e], order 2: [-1, e+1], order 3: [-2, e+1]).
template <int O, int DIM>
struct TileWin {
  static constexpr int LO = (O == 3) ? -2 : -1;
  static constexpr int R = (O == 3) ? 4 : (O == 2 ? 3 : 2);
  int o[3];
  int W[3];
  int size;
  int c0[3], e[3];

  __device__ __forceinline__ explicit TileWin(const TileBox& tb) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      c0[d] = tb.c0[d];
      e[d] = tb.e[d];
      if (d < DIM) {
        o[d] = tb.c0[d] + LO;
        W[d] = tb.e[d] + R;
      } else {
        o[d] = 0;
        W[d] = 1;
      }
    }
    size = W[0] * W[1] * W[2];
  }

  __host__ __device__ static int max_size(const KBins& kb) {
    int s = 1;
    for (int d = 0; d < 3; ++d) s *= (d < DIM) ? kb.T[d] + R : 1;
    return s;
  }

  // A particle whose cell lies in the tile has its whole stencil inside the window.
  __device__ __forceinline__ bool fits(const PartPrep<O, DIM>& p) const {
    bool in = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) in = in && p.cell[d] >= c0[d] && p.cell[d] < c0[d] + e[d];
    return in;
  }

  __device__ __forceinline__ int index(int c, int mx, int my, int mz) const {
    return c * size + ((mz - o[2]) * W[1] + (my - o[1])) * W[0] + (mx - o[0]);
  }

  __device__ __forceinline__ bool fits_cell(const int* cell) const {
    bool in = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) in = in && cell[d] >= c0[d] && cell[d] < c0[d] + e[d];
    return in;
  }
};

// Per-wave mover buffer in LDS: movers are appended with a ballot and a lane prefix
// count and copied to the global list, with one global atomic per flush, when it fills
// and at the end of the tile (usually once per tile: the list counter is contended).
constexpr int MBUF = 128;

// Workgroups appended to a one-workgroup-per-tile launch that write the outputs of the
// slots past the last bin (gaps) with a grid-stride loop; one workgroup alone would take
// longer than the tiles for large slack.
constexpr int TAIL_BLOCKS = 64;

struct MoverBuf {
  int32_t* slot;
  int32_t* oldb;
  int32_t* newb;
  int cnt;  // wave-uniform
};

__device__ __forceinline__ void mb_flush(MoverBuf& mb, const KBins& B) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (mb.cnt > 0) {
    const int lane = __lane_id();
    int base = 0;
    if (lane == 0) base = atomicAdd(&B.ctr[CTR_NMOV], mb.cnt);
    base = __shfl(base, 0);
    int drop = 0;
    for (int i = lane; i < mb.cnt; i += PIC_WAVE) {
      const int e = base + i;
      if (e < B.max_movers) {
        B.mv_slot[e] = mb.slot[i];
        B.mv_old[e] = mb.oldb[i];
        B.mv_new[e] = mb.newb[i];
      } else {
        ++drop;
      }
    }
    if (drop) atomicAdd(&B.ctr[CTR_NDROP], drop);
  }
  mb.cnt = 0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Every lane of the wave must call it (uniform control flow).
__device__ __forceinline__ void mb_append(MoverBuf& mb, const KBins& B, bool pred, int slot,
                                          int ob, int nb) {
  const unsigned long long m = __ballot(pred);
  if (m == 0ull) return;
  const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                             __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
  if (pred) {
    mb.slot[mb.cnt + rank] = slot;
    mb.oldb[mb.cnt + rank] = ob;
    mb.newb[mb.cnt + rank] = nb;
  }
  mb.cnt += (int)__popcll(m);
  if (mb.cnt > MBUF - PIC_WAVE) mb_flush(mb, B);
}

// Bytes of LDS in front of the window: bin offsets (nb + 1) and lengths (nb).
__host__ __device__ __forceinline__ size_t tile_smem_head(const KBins& kb) {
  size_t nb = (size_t)kb.T[0] * kb.T[1] * kb.T[2];
  return ((2 * nb + 1) * sizeof(int32_t) + 15) & ~(size_t)15;
}

// Bin (0..nb-1) of slot s, given the tile's bin offsets s_off[0..nb] with s in
// [s_off[0], s_off[nb]).
__device__ __forceinline__ int slot_bin(const int32_t* s_off, int nb, int s) {
  int lo = 0, hi = nb;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (s_off[mid] <= s) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Store the tile's window to its slab of the window scratch (plain coalesced stores);
// k_halo_tile then adds the overlapping windows of neighbouring tiles into J, so no
// global atomics are needed (and the sum is deterministic).
template <int O, int DIM>
__device__ __forceinline__ void store_window(const KBins& B, int tile, const TileWin<O, DIM>& tw,
                                             const float* win, int nthr, int tid) {
  float* dst = B.wscr + (int64_t)tile * 3 * B.wmax;
  for (int c = 0; c < 3; ++c)
    for (int i = tid; i < tw.size; i += nthr) dst[(int64_t)c * B.wmax + i] = win[c * tw.size + i];
}

// One patch of a batched launch, as the persistent kernels read it.
struct BatchPatch {
  KGrid G;
  KBins B;
  KPart P;
  float* J[3];
  double dt;
};

// Batched launches (deposit_cell.hip, deposit.hip).
size_t cell_smem_bytes(int order, int dim, const KBins& kb);
int batched_blocks_per_cu(size_t smem);
void batched_cell_launch(const BatchPatch* pd, const int2* items, int nitems, int* queue,
                         int blocks, size_t smem, unsigned flags, hipStream_t s);
void batched_prologue_launch(const BatchPatch* pd, int npatch, int64_t max_nodes, int* queue,
                             unsigned flags, hipStream_t s);
size_t halo_smem_bytes(const KBins& kb);
int halo_row_tiles();   // tiles along x summed by one window-sum workgroup
void batched_halo_tile_launch(const BatchPatch* pd, const int2* items, int nitems, size_t smem,
                              hipStream_t s);

// Charge density on the per-cell path (deposit_cell.hip) and its window sum (deposit.hip).
bool deposit_rho_cell_launch(const KGrid& G, const KPart& P, pic_bins* b, float* rho,
                             hipStream_t s);
void halo_rho_launch(const KGrid& G, pic_bins* b, float* rho, hipStream_t s);

// Path selection and the per-cell paths (deposit_cell.hip).
int choose_path(const KGrid& G, const pic_bins* b);
bool deposit_cell_launch(const KGrid& G, const KPart& P, pic_bins* b, float* J0, float* J1,
                         float* J2, int path, unsigned flags, double dt, hipStream_t s);
