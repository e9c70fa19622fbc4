// Cell-sorted particle bins on the GPU (Sec. 4.3-4.4 of the paper, re-designed).
//
// The paper keeps a gapped packed-memory array of particle indices per tile and moves
// payload only at global sorts. Here every cell owns a bin of slots [off[b], off[b+1])
// in the particle arrays themselves; its first len[b] slots hold its particles (moved
// physically, so deposition reads them with coalesced loads) and the rest are gaps
// (id = -1, w = 0). Bins are laid out tile by tile, so a tile's particles are one
// contiguous slot range.
//
// FULL (GlobalSortParticlesByCell, Alg. 1): histogram -> per-bin capacity len + slack
//   -> exclusive scan -> scatter into staging -> per-bin sort by id -> copy back.
// INCREMENTAL (Sec. 4.3.1-4.3.2): movers are (slot, old bin, new bin) entries found
//   with a wave ballot (fused into deposition, or by k_detect). Insert: an atomic slot
//   reservation in the destination bin's gaps and a payload copy; the source slot
//   becomes a gap (O(1) delete). Compact: each touched bin fills its holes from its top
//   entries (swap-with-last). A full destination bin flags its tile; a flagged tile is
//   rebuilt with fresh, uniformly spread gaps (local rebuild, Sec. 4.3.2) and the mover
//   stays in its old bin until the next rebin (deposition handles such particles).
#include <algorithm>

#include "pic_host.h"

__global__ void k_zero_i32(int32_t* __restrict__ p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0;
}

static void zero_i32(int32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_zero_i32, dim3(blocks), dim3(256), 0, s, p, n);
}

static unsigned grid_for(int64_t n, int64_t cap = 16384) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap));
}

// ---------------------------------------------------------------------------------
// Exclusive scan of int32 (2048 elements per block of 256 threads, recursive sums).
__global__ __launch_bounds__(256) void k_scan_blocks(int32_t* __restrict__ data, int64_t n,
                                                     int32_t* __restrict__ sums) {
  __shared__ int32_t s_tot[256];
  const int64_t base = (int64_t)blockIdx.x * 2048 + threadIdx.x * 8;
  int32_t v[8];
  int32_t run = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int64_t i = base + k;
    int32_t x = i < n ? data[i] : 0;
    v[k] = run;
    run += x;
  }
  s_tot[threadIdx.x] = run;
  __syncthreads();
  // inclusive scan of thread totals (Hillis-Steele in LDS)
  for (int off = 1; off < 256; off <<= 1) {
    int32_t t = threadIdx.x >= off ? s_tot[threadIdx.x - off] : 0;
    __syncthreads();
    s_tot[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t excl = threadIdx.x ? s_tot[threadIdx.x - 1] : 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int64_t i = base + k;
    if (i < n) data[i] = v[k] + excl;
  }
  if (threadIdx.x == 255 && sums) sums[blockIdx.x] = s_tot[255];
}

__global__ __launch_bounds__(256) void k_scan_add(int32_t* __restrict__ data, int64_t n,
                                                  const int32_t* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * 2048;
  const int32_t add = sums[blockIdx.x];
  for (int k = threadIdx.x; k < 2048; k += 256) {
    int64_t i = base + k;
    if (i < n) data[i] += add;
  }
}

static void scan_rec(pic_bins* b, int32_t* data, int64_t n, int level, hipStream_t s) {
  int64_t nb = (n + 2047) / 2048;
  if (nb <= 1) {
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(256), 0, s, data, n, (int32_t*)nullptr);
    return;
  }
  int32_t* sums = b->scan_tmp[level];
  hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(256), 0, s, data, n, sums);
  scan_rec(b, sums, nb, level + 1, s);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(256), 0, s, data, n, sums);
}

void scan_exclusive_i32(pic_bins* b, int32_t* data, int64_t n, hipStream_t s) {
  scan_rec(b, data, n, 0, s);
}

// ---------------------------------------------------------------------------------
// One particle's payload. Copies load all eight fields before storing any: the arrays may
// alias (source and destination are often the same particle arrays), so a store placed
// between two loads would keep the second load waiting for the first store.
struct Payload {
  double x, y, z;
  float ux, uy, uz, w;
  int32_t id;
};

__device__ __forceinline__ Payload load_slot(const KPart& S, int s) {
  return Payload{S.x[s], S.y[s], S.z[s], S.ux[s], S.uy[s], S.uz[s], S.w[s], S.id[s]};
}

__device__ __forceinline__ void store_slot(const KPart& D, int d, const Payload& p) {
  D.x[d] = p.x;
  D.y[d] = p.y;
  D.z[d] = p.z;
  D.ux[d] = p.ux;
  D.uy[d] = p.uy;
  D.uz[d] = p.uz;
  D.w[d] = p.w;
  D.id[d] = p.id;
}

__device__ __forceinline__ void copy_slot(const KPart& D, int d, const KPart& S, int s) {
  const Payload p = load_slot(S, s);
  store_slot(D, d, p);
}

// A gap slot is marked by its id and weight alone (every kernel tests the id before it
// reads a slot's payload), so turning a slot into a gap touches two arrays, not eight.
__device__ __forceinline__ void set_gap(const KPart& D, int d) {
  D.w[d] = 0.0f;
  D.id[d] = PIC_INVALID_ID;
}

// Gap slot written in every array, for passes that rewrite whole slot ranges: their lines
// are then written in full and never read back to merge a partial write.
__device__ __forceinline__ void set_gap_full(const KPart& D, int d) {
  D.x[d] = 0.0;
  D.y[d] = 0.0;
  D.z[d] = 0.0;
  D.ux[d] = 0.0f;
  D.uy[d] = 0.0f;
  D.uz[d] = 0.0f;
  D.w[d] = 0.0f;
  D.id[d] = PIC_INVALID_ID;
}

__device__ __forceinline__ void swap_slots(const KPart& D, int a, int c) {
  const Payload pa = load_slot(D, a), pc = load_slot(D, c);
  store_slot(D, a, pc);
  store_slot(D, c, pa);
}

// Sort slots [o, o + n) by id (insertion sort on the payload; bins are small).
__device__ void sort_range_by_id(const KPart& D, int o, int n) {
  for (int i = 1; i < n; ++i) {
    int j = i;
    while (j > 0 && D.id[o + j - 1] > D.id[o + j]) {
      swap_slots(D, o + j - 1, o + j);
      --j;
    }
  }
}

template <int DIM>
__device__ __forceinline__ int32_t bin_of_pos(const KGrid& G, const KBins& B, double x, double y,
                                              double z, uint32_t& bad) {
  float f;
  int i = to_cell(x, G.x0[0], G.inv_dx[0], G.n[0], f, bad);
  int j = to_cell(y, G.x0[1], G.inv_dx[1], G.n[1], f, bad);
  int k = DIM == 3 ? to_cell(z, G.x0[2], G.inv_dx[2], G.n[2], f, bad) : 0;
  if (i < 0 || j < 0 || k < 0) return -1;
  return bin_of_cell(G.n, B.T, i, j, k);
}

// ---- FULL ------------------------------------------------------------------------
// Runs of equal keys among the 64 lanes of a wave (consecutive slots): the run's first lane,
// this lane's position in the run and the run length. Between global sorts most particles
// still sit in their bin, so consecutive slots mostly share a bin and one atomic per run
// replaces one per particle.
__device__ __forceinline__ void wave_runs(int32_t key, int& head, int& pos, int& len) {
  const int lane = __lane_id();
  const int32_t prev = __shfl_up(key, 1);
  const bool is_head = lane == 0 || prev != key;
  const unsigned long long hm = __ballot(is_head);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  head = 63 - __builtin_clzll(hm & upto);
  const unsigned long long above = hm & ~upto;
  const int next = above ? __builtin_ctzll(above) : 64;
  pos = lane - head;
  len = next - head;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* s_part) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x / PIC_WAVE;
  __syncthreads();
  if (__lane_id() == 0) s_part[w] = v;
  __syncthreads();
  T t = 0;
  for (int i = 0; i < (int)(blockDim.x / PIC_WAVE); ++i) t += s_part[i];
  return t;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_full_count(KGrid G, KBins B, KPart P,
                                                    int32_t* __restrict__ sbin) {
  __shared__ int32_t s_part[4];
  uint32_t bad = 0;
  int32_t counted = 0;
  const int stride = gridDim.x * blockDim.x;
  // uniform trip count: every lane reaches the wave-level run detection
  for (int base = blockIdx.x * blockDim.x; base < P.nslots; base += stride) {
    const int s = base + threadIdx.x;
    int32_t bn = -1;
    if (s < P.nslots && P.id[s] != PIC_INVALID_ID)
      bn = bin_of_pos<DIM>(G, B, P.x[s], P.y[s], DIM == 3 ? P.z[s] : 0.0, bad);
    if (s < P.nslots) sbin[s] = bn;
    int head, pos, len;
    wave_runs(bn, head, pos, len);
    if (bn >= 0 && pos == 0) atomicAdd(&B.len[bn], len);
    counted += bn >= 0 ? 1 : 0;
  }
  const int32_t tot = block_sum(counted, s_part);
  if (threadIdx.x == 0 && tot) atomicAdd(&B.ctr[CTR_TOTAL], tot);
  if (bad) atomicOr(B.err, bad);
}

__global__ __launch_bounds__(256) void k_full_extra(KBins B, double slack,
                                                    unsigned long long* desired) {
  __shared__ unsigned long long s_part[4];
  unsigned long long acc = 0;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B.nbins; b += gridDim.x * blockDim.x) {
    int32_t e = (int32_t)ceil(slack * (double)B.len[b]);
    B.ins_cnt[b] = e;
    acc += (unsigned long long)e;
  }
  const unsigned long long tot = block_sum(acc, s_part);
  if (threadIdx.x == 0 && tot) atomicAdd(desired, tot);
}

__global__ __launch_bounds__(256) void k_full_caps(KBins B, int32_t nslots,
                                                   const unsigned long long* desired) {
  const int64_t total = B.ctr[CTR_TOTAL];
  const int64_t free_slots = (int64_t)nslots - total;
  const unsigned long long want = *desired;
  const bool scale = (unsigned long long)std::max<int64_t>(free_slots, 0) < want;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= B.nbins; b += gridDim.x * blockDim.x) {
    if (b == B.nbins) {
      B.off[b] = 0;
      continue;
    }
    int64_t e = B.ins_cnt[b];
    if (scale) e = want ? (int64_t)((double)e * (double)free_slots / (double)want) : 0;
    B.off[b] = B.len[b] + (int32_t)e;
  }
}

// Payload of every counted particle to its bin in the staging arrays; the rank inside the
// bin comes from one atomic per run of equal bins.
__global__ __launch_bounds__(256) void k_full_scatter(KBins B, KPart P, KPart S,
                                                      const int32_t* __restrict__ sbin) {
  const int stride = gridDim.x * blockDim.x;
  for (int base = blockIdx.x * blockDim.x; base < P.nslots; base += stride) {
    const int s = base + threadIdx.x;
    const int32_t bn = s < P.nslots ? sbin[s] : -1;
    int head, pos, len;
    wave_runs(bn, head, pos, len);
    int r = 0;
    if (bn >= 0 && pos == 0) r = atomicAdd(&B.ins_cnt[bn], len);
    r = __shfl(r, head);
    if (bn >= 0) copy_slot(S, B.off[bn] + r + pos, P, s);
  }
}

// Final placement in two passes. Ranks, one thread per bin: the staged particle j of bin b
// goes to its rank by id inside the bin (a deterministic order whatever order the
// scatter's atomics produced); src[o + rank] = o + j, and -1 on the bin's gap slots.
__global__ __launch_bounds__(256) void k_full_rank(KBins B, KPart S, int32_t* __restrict__ src) {
  const int stride = gridDim.x * blockDim.x;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B.nbins; b += stride) {
    const int o = B.off[b], n = B.len[b], cap = B.off[b + 1] - o;
    if (n <= 16) {
      int32_t ids[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) ids[k] = k < n ? S.id[o + k] : INT32_MAX;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        if (j < n) {
          int r = 0;
#pragma unroll
          for (int k = 0; k < 16; ++k) r += ids[k] < ids[j] ? 1 : 0;
          src[o + r] = o + j;
        }
      }
    } else {
      for (int j = 0; j < n; ++j) {
        const int32_t idj = S.id[o + j];
        int r = 0;
        for (int k = 0; k < n; ++k) r += S.id[o + k] < idj ? 1 : 0;
        src[o + r] = o + j;
      }
    }
    for (int j = n; j < cap; ++j) src[o + j] = -1;
    B.ins_cnt[b] = 0;
    B.out_flag[b] = 0;
  }
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  for (int t = tid; t < B.ntiles; t += stride) B.tile_flag[t] = 0;
}

// Copy, lanes = destination slots (coalesced writes): particle arrays <- staged payload,
// gaps where src is -1 and past the last bin.
__global__ __launch_bounds__(256) void k_full_place(KBins B, KPart P, KPart S,
                                                    const int32_t* __restrict__ src) {
  const int used = B.off[B.nbins];
  for (int d = blockIdx.x * blockDim.x + threadIdx.x; d < P.nslots; d += gridDim.x * blockDim.x) {
    const int j = d < used ? src[d] : -1;
    if (j >= 0) copy_slot(P, d, S, j);
    else set_gap_full(P, d);
  }
}

__global__ void k_full_finish(KBins B) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    B.ctr[CTR_NVALID] = B.ctr[CTR_TOTAL];
    B.ctr[CTR_TOTAL] = 0;
    B.ctr[CTR_NMOV] = 0;
    B.ctr[CTR_NMOV_LAST] = 0;
  }
}

void rebin_full(pic_bins* b, const KGrid& G, const KPart& P, hipStream_t s) {
  KBins& B = b->kb;
  const int64_t ns = b->nslots;
  zero_i32(B.len, B.nbins, s);
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, (int32_t*)&b->dctr->desired, (int64_t)2);
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, B.ctr + CTR_TOTAL, (int64_t)1);
  if (ns > 0) {
    if (G.dim == 3)
      hipLaunchKernelGGL(k_full_count<3>, dim3(grid_for(ns, 4096)), dim3(256), 0, s, G, B, P, b->sbin);
    else
      hipLaunchKernelGGL(k_full_count<2>, dim3(grid_for(ns, 4096)), dim3(256), 0, s, G, B, P, b->sbin);
  }
  hipLaunchKernelGGL(k_full_extra, dim3(grid_for(B.nbins, 2048)), dim3(256), 0, s, B, b->slack,
                     &b->dctr->desired);
  hipLaunchKernelGGL(k_full_caps, dim3(grid_for(B.nbins + 1)), dim3(256), 0, s, B, (int32_t)ns,
                     &b->dctr->desired);
  scan_exclusive_i32(b, B.off, B.nbins + 1, s);
  zero_i32(B.ins_cnt, B.nbins, s);
  if (ns > 0)
    hipLaunchKernelGGL(k_full_scatter, dim3(grid_for(ns, 4096)), dim3(256), 0, s, B, P, b->scratch,
                       b->sbin);
  hipLaunchKernelGGL(k_full_rank, dim3(grid_for(std::max<int64_t>(B.nbins, B.ntiles))),
                     dim3(256), 0, s, B, b->scratch, b->sbin);
  if (ns > 0)
    hipLaunchKernelGGL(k_full_place, dim3(grid_for(ns, 8192)), dim3(256), 0, s, B, P, b->scratch,
                       b->sbin);
  hipLaunchKernelGGL(k_full_finish, dim3(1), dim3(64), 0, s, B);
}

// ---- INCREMENTAL -------------------------------------------------------------------
// Mover detection without deposition: one workgroup per tile, coalesced slot loop.
template <int DIM>
__global__ __launch_bounds__(256) void k_detect(KGrid G, KBins B, KPart P) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileBox tb = tile_box(G.n, B.T, B.nt, blockIdx.x);
  int32_t* s_off = (int32_t*)smem_raw;
  int32_t* s_len = s_off + tb.nb + 1;
  for (int i = threadIdx.x; i <= tb.nb; i += blockDim.x) s_off[i] = B.off[tb.b0 + i];
  for (int i = threadIdx.x; i < tb.nb; i += blockDim.x) s_len[i] = B.len[tb.b0 + i];
  __syncthreads();
  const int S0 = s_off[0], S1 = s_off[tb.nb];
  uint32_t bad = 0;
  for (int base = S0; base < S1; base += blockDim.x) {
    int s = base + threadIdx.x;
    bool mv = false;
    int lb = 0;
    int32_t nb = -1;
    if (s < S1) {
      int lo = 0, hi = tb.nb;
      while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (s_off[mid] <= s) lo = mid;
        else hi = mid;
      }
      lb = lo;
      if (s < s_off[lb] + s_len[lb]) {
        nb = bin_of_pos<DIM>(G, B, P.x[s], P.y[s], DIM == 3 ? P.z[s] : 0.0, bad);
        mv = nb >= 0 && nb != tb.b0 + lb;
      }
    }
    int e = wave_append(mv, &B.ctr[CTR_NMOV]);
    if (mv) {
      if (e < B.max_movers) {
        B.mv_slot[e] = s;
        B.mv_old[e] = tb.b0 + lb;
        B.mv_new[e] = nb;
      } else {
        atomicAdd(&B.ctr[CTR_NDROP], 1);
      }
    }
  }
  if (bad) atomicOr(B.err, bad);
}

__global__ __launch_bounds__(256) void k_insert(KBins B, KPart P, const int32_t* __restrict__ bin_cell,
                                                int nx, int ny) {
  const int nmov = min(B.ctr[CTR_NMOV], B.max_movers);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nmov; e += gridDim.x * blockDim.x) {
    const int s = B.mv_slot[e], ob = B.mv_old[e], nb = B.mv_new[e];
    const Payload pl = load_slot(P, s);   // in flight while the destination is claimed
    const int k = atomicAdd(&B.ins_cnt[nb], 1);
    const int pos = B.len[nb] + k;
    const int cap = B.off[nb + 1] - B.off[nb];
    const bool fits = pos < cap;
    if (fits) {
      store_slot(P, B.off[nb] + pos, pl);
      set_gap(P, s);
      B.out_flag[ob] = 1;     // the source bin has a hole (plain store: every writer writes 1)
    } else {
      int c = bin_cell[nb];
      int i = c % nx, j = (c / nx) % ny, kk = c / (nx * ny);
      atomicAdd(&B.tile_flag[tile_of_cell(B.T, B.nt, i, j, kk)], 1);
    }
    // one atomic per wave on the shared overflow counter (tens of thousands of
    // same-address atomics per step would serialise in the L2)
    const unsigned long long m = __ballot(!fits);
    if (m && __lane_id() == __ffsll((long long)m) - 1)
      atomicAdd(&B.ctr[CTR_NOVF], (int)__popcll(m));
  }
}

// Compaction of every bin that lost or gained particles: holes (gap slots) in the old dense
// prefix [0, L) are filled, in slot order, by the valid entries at or above the new length
// (the prefix's tail, then the inserted particles ordered by id): swap-with-last of the
// paper's delete, with one payload copy per hole. The bin's hole count is read from the
// ids themselves.
__global__ __launch_bounds__(256) void k_compact(KBins B, KPart P) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B.nbins; b += gridDim.x * blockDim.x) {
    const int outf = B.out_flag[b], ins = B.ins_cnt[b];
    if (outf == 0 && ins == 0) continue;
    const int o = B.off[b];
    const int L = B.len[b];
    const int cap = B.off[b + 1] - o;
    const int I = min(ins, cap - L);
    if (I >= 2) sort_range_by_id(P, o + L, I);
    const int total = L + I;
    if (outf == 0) {
      // nothing left: no holes, the inserted particles extend the dense prefix
      B.len[b] = total;
    } else if (total <= 16) {
      // ids read at once (independent loads), holes and sources as bit masks
      int32_t ids[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) ids[k] = k < L ? P.id[o + k] : 0;
      unsigned gaps = 0u;
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < L && ids[k] == PIC_INVALID_ID) gaps |= 1u << k;
      const int nl = total - __builtin_popcount(gaps);
      // holes below nl; sources: valid entries at or above nl (inserted ones are valid)
      const unsigned below = nl >= 32 ? ~0u : ((1u << nl) - 1u);
      const unsigned all = total >= 32 ? ~0u : ((1u << total) - 1u);
      unsigned holes = gaps & below;
      unsigned srcs = all & ~below & ~gaps;
      while (holes && srcs) {
        const int h = __builtin_ctz(holes), t = __builtin_ctz(srcs);
        copy_slot(P, o + h, P, o + t);
        set_gap(P, o + t);
        holes &= holes - 1u;
        srcs &= srcs - 1u;
      }
      B.len[b] = nl;
    } else {
      int out = 0;
      for (int i = 0; i < L; ++i) out += P.id[o + i] == PIC_INVALID_ID ? 1 : 0;
      const int nl = total - out;
      int top = nl;
      for (int i = 0; i < nl; ++i) {
        if (P.id[o + i] != PIC_INVALID_ID) continue;
        while (top < total && P.id[o + top] == PIC_INVALID_ID) ++top;
        if (top >= total) break;
        copy_slot(P, o + i, P, o + top);
        set_gap(P, o + top);
        ++top;
      }
      B.len[b] = nl;
    }
    B.out_flag[b] = 0;
    B.ins_cnt[b] = 0;
  }
}

// Local rebuild of flagged tiles: the tile's slots are redistributed with the free slots
// spread uniformly over its cells (order inside a bin is kept).
// A tile is rebuilt once at least max(2, cells / 32) of its inserts overflowed in one
// rebin: a single overflow leaves one particle in its old bin (deposited exactly, retried
// next rebin), which is far cheaper than moving the whole tile.
__global__ __launch_bounds__(256) void k_rebuild(KGrid G, KBins B, KPart P, KPart S) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int t = blockIdx.x;
  const int nflag = B.tile_flag[t];
  if (nflag == 0) return;
  const TileBox tb = tile_box(G.n, B.T, B.nt, t);
  if (nflag < max(2, tb.nb / 32)) {
    __syncthreads();
    if (threadIdx.x == 0) B.tile_flag[t] = 0;
    return;
  }
  int32_t* s_off = (int32_t*)smem_raw;     // old offsets, nb + 1
  int32_t* s_len = s_off + tb.nb + 1;      // lengths, nb
  int32_t* s_new = s_len + tb.nb;          // new offsets, nb + 1
  __shared__ int32_t s_part[256];
  for (int i = threadIdx.x; i <= tb.nb; i += blockDim.x) s_off[i] = B.off[tb.b0 + i];
  for (int i = threadIdx.x; i < tb.nb; i += blockDim.x) s_len[i] = B.len[tb.b0 + i];
  __syncthreads();
  const int S0 = s_off[0], S1 = s_off[tb.nb];
  // particles in the tile
  int cnt = 0;
  for (int i = threadIdx.x; i < tb.nb; i += blockDim.x) cnt += s_len[i];
  s_part[threadIdx.x] = cnt;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) s_part[threadIdx.x] += s_part[threadIdx.x + off];
    __syncthreads();
  }
  const int N = s_part[0];
  const int free_slots = (S1 - S0) - N;
  const int per = free_slots / tb.nb, rem = free_slots % tb.nb;
  __syncthreads();
  // new offsets: serial chunks per thread, then a scan of chunk totals
  const int chunk = (tb.nb + blockDim.x - 1) / blockDim.x;
  const int i0 = threadIdx.x * chunk, i1 = min(tb.nb, i0 + chunk);
  int run = 0;
  for (int i = i0; i < i1; ++i) run += s_len[i] + per + (i < rem ? 1 : 0);
  s_part[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int v = threadIdx.x >= off ? s_part[threadIdx.x - off] : 0;
    __syncthreads();
    s_part[threadIdx.x] += v;
    __syncthreads();
  }
  int acc = S0 + (threadIdx.x ? s_part[threadIdx.x - 1] : 0);
  for (int i = i0; i < i1; ++i) {
    s_new[i] = acc;
    acc += s_len[i] + per + (i < rem ? 1 : 0);
  }
  if (threadIdx.x == 0) s_new[tb.nb] = S1;
  // stage the tile's slots as they are, then write every slot of the new layout from the
  // staging copy (lanes = slots in both passes; the new bin of a slot by binary search)
  for (int s = S0 + threadIdx.x; s < S1; s += blockDim.x) copy_slot(S, s, P, s);
  __threadfence_block();
  __syncthreads();
  for (int d = S0 + threadIdx.x; d < S1; d += blockDim.x) {
    int lo = 0, hi = tb.nb;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_new[mid] <= d) lo = mid;
      else hi = mid;
    }
    const int k = d - s_new[lo];
    if (k < s_len[lo]) copy_slot(P, d, S, s_off[lo] + k);
    else set_gap_full(P, d);
  }
  for (int i = threadIdx.x; i < tb.nb; i += blockDim.x) B.off[tb.b0 + i] = s_new[i];
  if (threadIdx.x == 0) {
    B.tile_flag[t] = 0;
    atomicAdd(&B.ctr[CTR_NREB], 1);
  }
}

void rebin_incremental(pic_bins* b, const KGrid& G, const KPart& P, hipStream_t s) {
  KBins& B = b->kb;
  const size_t head = (((size_t)2 * B.T[0] * B.T[1] * B.T[2] + 1) * sizeof(int32_t) + 15) & ~(size_t)15;
  if (!b->movers_fresh) {
    reset_movers(b, s);
    if (G.dim == 3)
      hipLaunchKernelGGL(k_detect<3>, dim3(B.ntiles), dim3(256), head, s, G, B, P);
    else
      hipLaunchKernelGGL(k_detect<2>, dim3(B.ntiles), dim3(256), head, s, G, B, P);
  }
  hipLaunchKernelGGL(k_insert, dim3(grid_for(B.max_movers, 4096)), dim3(256), 0, s, B, P,
                     b->bin_cell, G.n[0], G.n[1]);
  hipLaunchKernelGGL(k_compact, dim3(grid_for(B.nbins)), dim3(256), 0, s, B, P);
  const size_t rb_smem = ((size_t)3 * B.T[0] * B.T[1] * B.T[2] + 2) * sizeof(int32_t);
  hipLaunchKernelGGL(k_rebuild, dim3(B.ntiles), dim3(256), rb_smem, s, G, B, P, b->scratch);
}

// ---- statistics and counters -------------------------------------------------------
// End of a rebin: the counters as they stand go to the snapshot block (which the host
// copies), then the per-rebin ones restart from zero for the next step.
__global__ void k_rebin_finish(KBins B, CtrBlock* c, CtrBlock* snap) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    B.ctr[CTR_NMOV_LAST] = min(B.ctr[CTR_NMOV], B.max_movers);
    c->cap_used = B.off[B.nbins];
    *snap = *c;
    B.ctr[CTR_NMOV] = 0;
    B.ctr[CTR_NDROP] = 0;
    B.ctr[CTR_NOVF] = 0;
    B.ctr[CTR_NREB] = 0;
  }
}

__global__ void k_reset_step(KBins B, int all) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    B.ctr[CTR_NMOV] = 0;
    B.ctr[CTR_NDROP] = 0;
    if (all) {
      B.ctr[CTR_NOVF] = 0;
      B.ctr[CTR_NREB] = 0;
    }
  }
}

void rebin_finish(pic_bins* b, hipStream_t s) {
  hipLaunchKernelGGL(k_rebin_finish, dim3(1), dim3(64), 0, s, b->kb, b->dctr, b->dctr + 1);
}

void reset_movers(pic_bins* b, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_step, dim3(1), dim3(64), 0, s, b->kb, 0);
}


