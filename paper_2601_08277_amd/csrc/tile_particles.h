// Dense enumeration of a tile's valid particles for the tiled gather-type kernels (field
// gather, push, adjoint gather): their threads run over particles, not over slots, of
// which a third are gaps at the usual slack.
#pragma once

#include "pic_internal.h"

// The valid particles of a tile, enumerated densely: pre[i] = particles in the tile's bins
// 0..i-1 (i = 0..nb, pre in LDS, `tmp` 256 ints of LDS), so that thread work can run over
// particles rather than slots (a third of the slots are gaps at the usual slack). Bins
// hold their particles in a dense prefix of their slots. Returns the count; ends with a
// barrier.
__device__ __forceinline__ int tile_valid_prefix(const KBins& B, const TileBox& tb, int* pre,
                                                 int* tmp) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = (tb.nb + nt - 1) / nt;
  const int lo = min(t * per, tb.nb), hi = min(lo + per, tb.nb);
  int sum = 0;
  for (int i = lo; i < hi; ++i) sum += B.len[tb.b0 + i];
  tmp[t] = sum;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {     // inclusive scan of the per-thread sums
    const int v = t >= off ? tmp[t - off] : 0;
    __syncthreads();
    tmp[t] += v;
    __syncthreads();
  }
  int run = t > 0 ? tmp[t - 1] : 0;
  for (int i = lo; i < hi; ++i) {
    pre[i] = run;
    run += B.len[tb.b0 + i];
  }
  if (t == nt - 1) pre[tb.nb] = tmp[nt - 1];
  __syncthreads();
  return pre[tb.nb];
}

// Slot of the j-th valid particle of the tile (0 <= j < pre[nb]).
__device__ __forceinline__ int tile_valid_slot(const KBins& B, const TileBox& tb, const int* pre,
                                               int j) {
  int lo = 0, hi = tb.nb;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= j) lo = mid;
    else hi = mid;
  }
  return B.off[tb.b0 + lo] + (j - pre[lo]);
}
