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
};

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

// Add the tile's window to J (float atomics: windows of neighbouring tiles overlap).
template <int O, int DIM>
__device__ __forceinline__ void flush_window(const KGrid& G, const TileWin<O, DIM>& tw,
                                             const float* win, float* const* J, int nthr,
                                             int tid) {
  const int W0 = tw.W[0], W01 = tw.W[0] * tw.W[1];
  for (int i = tid; i < 3 * tw.size; i += nthr) {
    float v = win[i];
    if (v == 0.0f) continue;
    int c = i / tw.size;
    int r = i - c * tw.size;
    int z = r / W01;
    int y = (r - z * W01) / W0;
    int x = r - z * W01 - y * W0;
    int ix = store_idx(G, 0, tw.o[0] + x);
    int iy = store_idx(G, 1, tw.o[1] + y);
    int iz = DIM == 3 ? store_idx(G, 2, tw.o[2] + z) : 0;
    if ((ix | iy | iz) < 0) continue;
    unsafeAtomicAdd(&J[c][((int64_t)iz * G.N[1] + iy) * G.N[0] + ix], v);
  }
}

// Path selection and the per-cell paths (deposit_cell.hip).
int choose_path(const KGrid& G, const pic_bins* b);
bool deposit_cell_launch(const KGrid& G, const KPart& P, pic_bins* b, float* J0, float* J1,
                         float* J2, int path, unsigned flags, double dt, hipStream_t s);
