// Per-cell deposition on VALU: the rhocell of Sec. 3.4 (Eq. 4) / Sec. 4.2.1 kept in
// registers.
//
// A workgroup owns one particle tile and has three waves, one per current component. It
// walks the tile in groups of 64 consecutive cells (one z-plane of an 8 x 8 x T tile).
// Bins are contiguous, so a group's particles are one contiguous slot range.
//  stage      all waves, lanes = slots, coalesced loads: position -> cell + float32 offset
//             (FP64 only here) and amplitude q W v_c; the fused drift and mover detection
//             (stage 1 of Alg. 2) also run here, once per particle, movers going to a
//             per-wave LDS buffer. Offsets and amplitudes go to LDS in cell order with
//             the gap slots skipped. A particle whose cell no longer matches its bin is
//             deposited at once through the per-particle path.
//  accumulate lanes = cells: the lane of wave c walks its cell's staged particles and
//             accumulates (amp_c s_x) (x) s_y (x) s_z of component c on the cell's padded
//             stencil window in registers (Eq. 4).
//  flush      once per cell and component, into the tile window in LDS (Eq. 5) with plain
//             read-add-write. The waves write different components, so they never share
//             a word. LDS float atomics cost about 190 cycles per wave instruction on
//             gfx950 (integer ones about 5) and are not used. The tile window then goes to
//             the window scratch; k_halo_sum adds neighbouring tiles into J.
// Staggered axes use a window one node wider than the stencil (the stencil of a particle
// in cell i starts at i + lo or i + lo + 1 depending on which half of the cell it is in);
// the extra node carries a zero weight.
#include "deposit_common.h"

template <int O, int DIM>
__host__ __device__ constexpr int cwin(int c, int d) {
  return d < DIM ? win_w(O, c == d) : 1;
}
template <int O, int DIM>
__host__ __device__ constexpr int csz(int c) {
  return cwin<O, DIM>(c, 0) * cwin<O, DIM>(c, 1) * cwin<O, DIM>(c, 2);
}
// Weights placed on the padded window: out[a] = w[a - s] (zero outside).
template <int O, int W>
__device__ __forceinline__ void pad_w(const float* w, int s, float* out) {
#pragma unroll
  for (int a = 0; a < W; ++a) {
    float v0 = (a <= O) ? w[a < O + 1 ? a : 0] : 0.0f;
    float v1 = (a >= 1 && a - 1 <= O) ? w[(a >= 1 && a - 1 <= O) ? a - 1 : 0] : 0.0f;
    out[a] = s ? v1 : v0;
  }
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
  return v;
}

constexpr int CV_GROUP = 64;    // cells per group (lanes)
constexpr int CV_CAP = 512;     // staged particles per round (gaps skipped)
constexpr int CV_MAPW = 1024;   // slots covered by one slot -> cell map window
constexpr int CV_WAVES = 3;     // one wave per current component

// LDS layout of one workgroup (bytes): bin offsets and lengths | tile window (3 comps)
// | staged offsets f[3][CAP] and amplitudes a[3][CAP] | slot -> cell map | mover buffers.
template <int O, int DIM>
struct CellLayout {
  size_t win_off, stage_off, map_off, mb_off, total;
  __host__ __device__ explicit CellLayout(const KBins& kb) {
    win_off = tile_smem_head(kb);
    stage_off = win_off + (((size_t)3 * TileWin<O, DIM>::max_size(kb) * sizeof(float) + 15) & ~(size_t)15);
    map_off = stage_off + (size_t)6 * CV_CAP * sizeof(float);
    mb_off = map_off + CV_MAPW;
    total = mb_off + (size_t)CV_WAVES * 3 * MBUF * sizeof(int32_t);
  }
};

struct CellGroup {
  int g0, gn;        // first tile-local bin, cells
  int S0, S1;        // slot range
  int n, st;         // this lane's cell: particles (valid slots), staged offset
  int ntot;          // particles of the group
};

// Stage the group's particles with staged index in [R0, R0 + CV_CAP): the three waves
// share the slot chunks, lanes = slots (coalesced loads).
template <int O, int DIM>
__device__ __forceinline__ void cv_stage(const KGrid& G, const KBins& B, const KPart& P,
                                         const TileBox& tb, const int32_t* s_off,
                                         const int32_t* s_len, const CellGroup& gr, int R0,
                                         float* sf, float* sa, int8_t* map, MoverBuf& mb,
                                         float* const* J, unsigned flags, double dt,
                                         uint32_t& bad) {
  const int wave = threadIdx.x / PIC_WAVE;
  const int lane = threadIdx.x % PIC_WAVE;
  const bool emit = flags & PIC_F_EMIT_MOVERS;
  const bool drift = flags & PIC_F_DRIFT;
  const int ex = tb.e[0], exy = tb.e[0] * tb.e[1];
  for (int lo = gr.S0; lo < gr.S1; lo += CV_MAPW) {
    const int hi = min(gr.S1, lo + CV_MAPW);
    __syncthreads();
    for (int i = threadIdx.x; i < hi - lo; i += blockDim.x) map[i] = -1;
    __syncthreads();
    if (wave == 0 && lane < gr.gn) {
      const int c = gr.g0 + lane;
      const int a = max(s_off[c], lo), b = min(s_off[c] + s_len[c], hi);
      for (int q = a; q < b; ++q) map[q - lo] = (int8_t)lane;
    }
    __syncthreads();
    for (int base = lo + wave * PIC_WAVE; base < hi; base += CV_WAVES * PIC_WAVE) {
      const int s = base + lane;
      int lc = s < hi ? (int)map[s - lo] : -1;
      const int lcs = lc < 0 ? 0 : lc;
      const int si = __shfl(gr.st, lcs) + (s - s_off[gr.g0 + lcs]) - R0;
      if (si < 0 || si >= CV_CAP) lc = -1;          // staged in another round
      const int lb = gr.g0 + lcs;
      PartPrep<O, DIM> p;
      double pos[3] = {0.0, 0.0, 0.0};
      float ux = 0.f, uy = 0.f, uz = 0.f;
      bool ok = false, mine = false;
      if (lc >= 0) {
        pos[0] = P.x[s];
        pos[1] = P.y[s];
        if (DIM == 3) pos[2] = P.z[s];
        ux = P.ux[s];
        uy = P.uy[s];
        uz = P.uz[s];
        const float w = P.w[s];
        ok = prep_cell<DIM>(G, pos[0], pos[1], pos[2], p.cell, p.f, bad);
        if (ok) {
          prep_amp(G.q, ux, uy, uz, w, p.amp);
          const int cz = lb / exy, cy = (lb - cz * exy) / ex, cxx = lb - cz * exy - cy * ex;
          mine = p.cell[0] == tb.c0[0] + cxx && p.cell[1] == tb.c0[1] + cy &&
                 (DIM == 2 || p.cell[2] == tb.c0[2] + cz);
        }
      }
      if (ok && !mine) {
        // stale particle (cell no longer matches its bin): exact per-particle path
        prep_shapes(p);
        scatter_particle(p, [&](int c, int mx, int my, int mz, float v) {
          int ix = store_idx(G, 0, mx), iy = store_idx(G, 1, my);
          int iz = DIM == 3 ? store_idx(G, 2, mz) : 0;
          if ((ix | iy | iz) < 0) {
            if (v != 0.0f) bad |= PIC_EF_STENCIL;
            return;
          }
          unsafeAtomicAdd(&J[c][((int64_t)iz * G.N[1] + iy) * G.N[0] + ix], v);
        });
      }
      if (lc >= 0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          sf[d * CV_CAP + si] = mine ? p.f[d] : 0.0f;
          sa[d * CV_CAP + si] = mine ? p.amp[d] : 0.0f;
        }
      }
      if (ok && drift) {
        drift_one<DIM>(G, pos, ux, uy, uz, dt);
        P.x[s] = pos[0];
        P.y[s] = pos[1];
        if (DIM == 3) P.z[s] = pos[2];
      }
      if (emit) {
        bool mv = false;
        int32_t nbn = -1;
        if (ok) {
          int c2[3];
          float f2[3];
          if (prep_cell<DIM>(G, pos[0], pos[1], pos[2], c2, f2, bad)) {
            nbn = bin_of_cell(G.n, B.T, c2[0], c2[1], c2[2]);
            mv = nbn != tb.b0 + lb;
          }
        }
        mb_append(mb, B, mv, s, tb.b0 + lb, nbn);
      }
    }
  }
  __syncthreads();
}

// Accumulate component C of the lane's cell from the staged particles [k0, k1).
template <int O, int DIM, int C>
__device__ __forceinline__ void cv_accumulate(int k0, int k1, const float* sf, const float* sa,
                                              float* acc) {
  constexpr int WX = cwin<O, DIM>(C, 0), WY = cwin<O, DIM>(C, 1), WZ = cwin<O, DIM>(C, 2);
  const int n = k1 - k0;
  const int nmax = wave_max(n);
  for (int k = 0; k < nmax; ++k) {
    const bool act = k < n;
    const int q = act ? k0 + k : 0;
    float f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) f[d] = sf[d * CV_CAP + q];
    const float amp = act ? sa[C * CV_CAP + q] : 0.0f;
    float wx[5], wy[5], wz[5];
    {
      float w[O + 1];
      int sh = shape_w<O, C == 0>(f[0], w);
      pad_w<O, WX>(w, sh, wx);
      sh = shape_w<O, C == 1>(f[1], w);
      pad_w<O, WY>(w, sh, wy);
      if constexpr (DIM == 3) {
        sh = shape_w<O, C == 2>(f[2], w);
        pad_w<O, WZ>(w, sh, wz);
      } else {
        wz[0] = 1.0f;
      }
    }
    float ax[5];
#pragma unroll
    for (int i = 0; i < WX; ++i) ax[i] = amp * wx[i];
#pragma unroll
    for (int iz = 0; iz < WZ; ++iz) {
#pragma unroll
      for (int iy = 0; iy < WY; ++iy) {
        const float t = wz[iz] * wy[iy];
#pragma unroll
        for (int ix = 0; ix < WX; ++ix) acc[(iz * WY + iy) * WX + ix] += ax[ix] * t;
      }
    }
  }
}

// Add component C of the lane's cell to the tile window with plain read-add-write. Within
// one instruction all lanes add at the same offset from their own (distinct) cells, so
// the 64 addresses differ; LDS executes a wave's instructions in order, and a compiler
// barrier keeps each read behind the previous write. When all cells of the group lie in
// one z-plane, two lanes can only meet on a node through offsets that differ in x or y, so
// the z-column of one (ix, iy) offset is read, added and written as a batch.
template <int O, int DIM, int C, bool ZBATCH>
__device__ __forceinline__ void cv_flush(const TileWin<O, DIM>& tw, const int* cc,
                                         const float* acc, float* win, bool own) {
  constexpr int WX = cwin<O, DIM>(C, 0), WY = cwin<O, DIM>(C, 1), WZ = cwin<O, DIM>(C, 2);
  const int lx = cc[0] + win_lo(O, C == 0);
  const int ly = cc[1] + win_lo(O, C == 1);
  const int lz = DIM == 3 ? cc[2] + win_lo(O, C == 2) : 0;
#pragma unroll
  for (int iy = 0; iy < WY; ++iy)
#pragma unroll
    for (int ix = 0; ix < WX; ++ix) {
      if constexpr (ZBATCH) {
        if (own) {
          float v[5];
#pragma unroll
          for (int iz = 0; iz < WZ; ++iz) v[iz] = win[tw.index(C, lx + ix, ly + iy, lz + iz)];
#pragma unroll
          for (int iz = 0; iz < WZ; ++iz)
            win[tw.index(C, lx + ix, ly + iy, lz + iz)] = v[iz] + acc[(iz * WY + iy) * WX + ix];
        }
        asm volatile("" ::: "memory");
      } else {
#pragma unroll
        for (int iz = 0; iz < WZ; ++iz) {
          if (own) {
            const int a = tw.index(C, lx + ix, ly + iy, lz + iz);
            win[a] = win[a] + acc[(iz * WY + iy) * WX + ix];
          }
          asm volatile("" ::: "memory");
        }
      }
    }
}

template <int O, int DIM>
__host__ __device__ constexpr int csz_max() {
  return csz<O, DIM>(0) > csz<O, DIM>(1) ? (csz<O, DIM>(0) > csz<O, DIM>(2) ? csz<O, DIM>(0) : csz<O, DIM>(2))
                                         : (csz<O, DIM>(1) > csz<O, DIM>(2) ? csz<O, DIM>(1) : csz<O, DIM>(2));
}

// One group: rounds of staging (all waves) and accumulation (wave c: component c), then
// the flush. The branches on the wave index are uniform within each wave and hold no
// barrier; every wave runs the same rounds, so all reach the same barriers.
template <int O, int DIM>
__device__ __forceinline__ void cv_group(const KGrid& G, const KBins& B, const KPart& P,
                                         const TileBox& tb, const TileWin<O, DIM>& tw,
                                         const int32_t* s_off, const int32_t* s_len,
                                         const CellGroup& gr, float* sf, float* sa, int8_t* map,
                                         MoverBuf& mb, float* win, float* const* J,
                                         unsigned flags, double dt, uint32_t& bad) {
  constexpr int NA = csz_max<O, DIM>();
  const int wave = threadIdx.x / PIC_WAVE;
  const int lane = threadIdx.x % PIC_WAVE;
  const bool own = lane < gr.gn;
  float acc[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) acc[i] = 0.0f;
  for (int R0 = 0; R0 < gr.ntot; R0 += CV_CAP) {
    cv_stage<O, DIM>(G, B, P, tb, s_off, s_len, gr, R0, sf, sa, map, mb, J, flags, dt, bad);
    const int k0 = min(max(gr.st, R0), R0 + CV_CAP) - R0;
    const int k1 = min(max(gr.st + gr.n, R0), R0 + CV_CAP) - R0;
    if (wave == 0) cv_accumulate<O, DIM, 0>(k0, k1, sf, sa, acc);
    else if (wave == 1) cv_accumulate<O, DIM, 1>(k0, k1, sf, sa, acc);
    else cv_accumulate<O, DIM, 2>(k0, k1, sf, sa, acc);
  }
  if (gr.ntot > 0) {
    const int ex = tb.e[0], exy = tb.e[0] * tb.e[1];
    const int cell = gr.g0 + (own ? lane : 0);
    int cc[3];
    cc[2] = cell / exy;
    cc[1] = (cell - cc[2] * exy) / ex;
    cc[0] = cell - cc[2] * exy - cc[1] * ex;
#pragma unroll
    for (int d = 0; d < 3; ++d) cc[d] += tb.c0[d];
    const bool plane = DIM == 3 && (gr.g0 / exy) == ((gr.g0 + gr.gn - 1) / exy);
    const bool o = own && gr.n > 0;
#define CV_FLUSH(C_)                                                     \
  if (plane) cv_flush<O, DIM, C_, true>(tw, cc, acc, win, o);            \
  else cv_flush<O, DIM, C_, false>(tw, cc, acc, win, o)
    if (wave == 0) { CV_FLUSH(0); }
    else if (wave == 1) { CV_FLUSH(1); }
    else { CV_FLUSH(2); }
#undef CV_FLUSH
  }
}

template <int O, int DIM>
__global__ __launch_bounds__(CV_WAVES * PIC_WAVE) void k_dep_cell_valu(
    KGrid G, KBins B, KPart P, float* __restrict__ J0, float* __restrict__ J1,
    float* __restrict__ J2, unsigned flags, double dt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const CellLayout<O, DIM> L(B);
  const TileBox tb = tile_box(G.n, B.T, B.nt, blockIdx.x);
  const TileWin<O, DIM> tw(tb);
  int32_t* s_off = (int32_t*)smem_raw;
  int32_t* s_len = s_off + tb.nb + 1;
  float* win = (float*)(smem_raw + L.win_off);
  float* sf = (float*)(smem_raw + L.stage_off);
  float* sa = sf + 3 * CV_CAP;
  int8_t* map = (int8_t*)(smem_raw + L.map_off);
  float* J[3] = {J0, J1, J2};
  const int wave = threadIdx.x / PIC_WAVE;
  const int lane = threadIdx.x % PIC_WAVE;
  int32_t* mbb = (int32_t*)(smem_raw + L.mb_off) + wave * 3 * MBUF;
  MoverBuf mb{mbb, mbb + MBUF, mbb + 2 * MBUF, 0};
  for (int i = threadIdx.x; i <= tb.nb; i += blockDim.x) s_off[i] = B.off[tb.b0 + i];
  for (int i = threadIdx.x; i < tb.nb; i += blockDim.x) s_len[i] = B.len[tb.b0 + i];
  for (int i = threadIdx.x; i < 3 * tw.size; i += blockDim.x) win[i] = 0.0f;
  __syncthreads();
  uint32_t bad = 0;
  for (int g0 = 0; g0 < tb.nb; g0 += CV_GROUP) {
    CellGroup gr;
    gr.g0 = g0;
    gr.gn = min(CV_GROUP, tb.nb - g0);
    gr.S0 = s_off[g0];
    gr.S1 = s_off[g0 + gr.gn];
    gr.n = lane < gr.gn ? s_len[g0 + lane] : 0;
    // exclusive scan of the cells' particle counts -> staged offsets
    int incl = gr.n;
#pragma unroll
    for (int off = 1; off < PIC_WAVE; off <<= 1) {
      const int t = __shfl_up(incl, off);
      if (lane >= off) incl += t;
    }
    gr.st = incl - gr.n;
    gr.ntot = __shfl(incl, PIC_WAVE - 1);
    cv_group<O, DIM>(G, B, P, tb, tw, s_off, s_len, gr, sf, sa, map, mb, win, J, flags, dt, bad);
  }
  if (flags & PIC_F_EMIT_MOVERS) mb_flush(mb, B);
  if (bad) atomicOr(B.err, bad);
  __syncthreads();
  store_window(B, blockIdx.x, tw, win, blockDim.x, threadIdx.x);
}

// ---------------------------------------------------------------------------------
bool deposit_mfma_launch(const KGrid& G, const KPart& P, pic_bins* b, float* J0, float* J1,
                         float* J2, int path, unsigned flags, double dt, hipStream_t s);

template <int O, int DIM>
static bool launch_cell_valu(const KGrid& G, const KPart& P, pic_bins* b, float* J0, float* J1,
                             float* J2, unsigned flags, double dt, hipStream_t s) {
  const size_t smem = CellLayout<O, DIM>(b->kb).total;
  if (smem > b->max_lds) return false;
  hipLaunchKernelGGL((k_dep_cell_valu<O, DIM>), dim3(b->kb.ntiles), dim3(CV_WAVES * PIC_WAVE), smem,
                     s, G, b->kb, P, J0, J1, J2, flags, dt);
  return true;
}

int choose_path(const KGrid& G, const pic_bins* b) {
  (void)G;
  (void)b;
  return PIC_PATH_CELL_VALU;
}

bool deposit_cell_launch(const KGrid& G, const KPart& P, pic_bins* b, float* J0, float* J1,
                         float* J2, int path, unsigned flags, double dt, hipStream_t s) {
  if (path == PIC_PATH_MFMA_BF16 || path == PIC_PATH_MFMA_FP16)
    return deposit_mfma_launch(G, P, b, J0, J1, J2, path, flags, dt, s);
#define CV(O_, D_) return launch_cell_valu<O_, D_>(G, P, b, J0, J1, J2, flags, dt, s)
  if (G.dim == 3) {
    if (G.order == 1) CV(1, 3); else if (G.order == 2) CV(2, 3); else CV(3, 3);
  } else {
    if (G.order == 1) CV(1, 2); else if (G.order == 2) CV(2, 2); else CV(3, 2);
  }
#undef CV
}
