// Per-cell deposition on VALU: the rhocell of Sec. 3.4 (Eq. 4) / Sec. 4.2.1 kept in
// registers.
//
// A workgroup owns one particle tile; its four waves own slabs of the tile's planes
// (z in 3D, y in 2D) and walk them in groups of up to 64 consecutive cells (one z-plane
// chunk in 3D). Bins are contiguous, so a group's particles are one contiguous slot range.
//  stage      lanes = slots, coalesced loads: position -> cell + float32 offset (FP64
//             only here), amplitude q W v_c; the fused drift and mover detection (stage 1
//             of Alg. 2) also run here, once per particle, movers going to a per-wave LDS
//             buffer. Offsets and amplitudes go to LDS. A particle whose cell no longer
//             matches its bin is deposited at once through the per-particle path.
//  accumulate lanes = cells: each lane walks its cell's staged particles and accumulates
//             the separable outer product (amp_c s_x) (x) s_y (x) s_z on the cell's padded
//             stencil window in registers (Eq. 4).
//  flush      once per cell, into the wave's own LDS sub-window (Eq. 5) with plain
//             read-add-write: within one instruction every lane adds at the same offset
//             from its own cell, so the 64 addresses differ. LDS float atomics cost about
//             190 cycles per wave instruction on gfx950 (integer ones about 5) and are not
//             used. At the end the four sub-windows are summed into the tile window slab
//             of the window scratch; k_halo_sum adds neighbouring tiles into J.
// Staggered axes use a window one node wider than the stencil (the stencil of a particle
// in cell i starts at i + lo or i + lo + 1 depending on which half of the cell it is in);
// the extra node carries a zero weight. Order 3 in 3D needs 3 x 80 accumulators; they are
// split over two passes (Jx, Jy then Jz) so a lane stays under 256 registers.
#include "deposit_common.h"

template <int O, int DIM>
__host__ __device__ constexpr int cwin(int c, int d) {
  return d < DIM ? win_w(O, c == d) : 1;
}
template <int O, int DIM>
__host__ __device__ constexpr int csz(int c) {
  return cwin<O, DIM>(c, 0) * cwin<O, DIM>(c, 1) * cwin<O, DIM>(c, 2);
}
// Offset of component c's accumulators (c = 3 gives the total).
template <int O, int DIM>
__host__ __device__ constexpr int acc_off(int c) {
  return (c > 0 ? csz<O, DIM>(0) : 0) + (c > 1 ? csz<O, DIM>(1) : 0) + (c > 2 ? csz<O, DIM>(2) : 0);
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

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int CV_GROUP = 64;    // cells per group (lanes)
constexpr int CV_CAP = 256;     // staged slots per wave per round
constexpr int CV_WAVES = 4;     // waves per workgroup (one slab each)

// Per-wave LDS area.
struct CellStage {
  float f[3][CV_CAP];
  float a[3][CV_CAP];
  int32_t mslot[MBUF], mold[MBUF], mnew[MBUF];
  int8_t map[CV_CAP];           // slot -> cell of the group (-1: gap)
};

struct CellCtx {
  int lane;
  int g0, gn;                   // group: first local bin, cells
};

// Stage slots [lo, hi) of the group: lanes = slots.
template <int O, int DIM, bool LAST>
__device__ __forceinline__ void cv_stage(const KGrid& G, const KBins& B, const KPart& P,
                                         const TileBox& tb, const int32_t* s_off,
                                         const int32_t* s_len, const CellCtx& cx, int lo, int hi,
                                         CellStage& st, MoverBuf& mb, float* const* J,
                                         unsigned flags, double dt, uint32_t& bad) {
  const int lane = cx.lane;
  const bool emit = LAST && (flags & PIC_F_EMIT_MOVERS);
  const bool drift = LAST && (flags & PIC_F_DRIFT);
  const int ex = tb.e[0], exy = tb.e[0] * tb.e[1];
  // slot -> cell map of this round
  for (int i = lane; i < CV_CAP; i += PIC_WAVE) st.map[i] = -1;
  wave_sync_lds();
  if (lane < cx.gn) {
    const int c = cx.g0 + lane;
    const int a = max(s_off[c], lo), b = min(s_off[c] + s_len[c], hi);
    for (int q = a; q < b; ++q) st.map[q - lo] = (int8_t)lane;
  }
  wave_sync_lds();
  for (int base = lo; base < hi; base += PIC_WAVE) {
    const int s = base + lane;
    const int k = s - lo;
    const int lc = s < hi ? (int)st.map[k] : -1;
    const int lb = cx.g0 + (lc < 0 ? 0 : lc);
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
    if (ok && !mine && LAST) {
      // stale particle: exact per-particle path (global atomics), all components, once
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
    if (s < hi) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        st.f[d][k] = mine ? p.f[d] : 0.0f;
        st.a[d][k] = mine ? p.amp[d] : 0.0f;
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
  wave_sync_lds();
}

// Accumulate components [CB, CE) of the group's cells from the staged slots [lo, hi).
template <int O, int DIM, int CB, int CE>
__device__ __forceinline__ void cv_accumulate(const int32_t* s_off, const int32_t* s_len,
                                              int cell, bool own, int lo, int hi,
                                              const CellStage& st, float* acc) {
  constexpr int A0 = acc_off<O, DIM>(CB);
  constexpr int WN = win_w(O, false), WS = win_w(O, true);
  int k0 = 0, k1 = 0;
  if (own) {
    k0 = max(s_off[cell], lo);
    k1 = min(s_off[cell] + s_len[cell], hi);
    if (k1 < k0) k1 = k0;
  }
  const int n = k1 - k0;
  const int nmax = wave_max(n);
  for (int k = 0; k < nmax; ++k) {
    const bool act = k < n;
    const int q = act ? k0 + k - lo : 0;
    float f[3], amp[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      f[d] = st.f[d][q];
      amp[d] = act ? st.a[d][q] : 0.0f;
    }
    float wnp[3][WN], wsp[3][WS];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      float w[O + 1];
      int sh = shape_w<O, false>(f[d], w);
      pad_w<O, WN>(w, sh, wnp[d]);
      if (d >= CB && d < CE) {
        sh = shape_w<O, true>(f[d], w);
        pad_w<O, WS>(w, sh, wsp[d]);
      }
    }
    if constexpr (DIM == 2) {
      wnp[2][0] = 1.0f;
      wsp[2][0] = 1.0f;
    }
#pragma unroll
    for (int c = CB; c < CE; ++c) {
      const int WX = cwin<O, DIM>(c, 0), WY = cwin<O, DIM>(c, 1), WZ = cwin<O, DIM>(c, 2);
      const float* wx = (c == 0) ? wsp[0] : wnp[0];
      const float* wy = (c == 1 && DIM >= 2) ? wsp[1] : wnp[1];
      const float* wz = (c == 2 && DIM == 3) ? wsp[2] : wnp[2];
      float ax[WS > WN ? WS : WN];
#pragma unroll
      for (int i = 0; i < WX; ++i) ax[i] = amp[c] * wx[i];
      const int base = acc_off<O, DIM>(c) - A0;
#pragma unroll
      for (int iz = 0; iz < WZ; ++iz) {
#pragma unroll
        for (int iy = 0; iy < WY; ++iy) {
          const float t = wz[iz] * wy[iy];
#pragma unroll
          for (int ix = 0; ix < WX; ++ix) acc[base + (iz * WY + iy) * WX + ix] += ax[ix] * t;
        }
      }
    }
  }
}

// Add the cell's accumulators to the wave's sub-window with plain read-add-write. In 3D
// all cells of a group lie in one z-plane, so two lanes can only meet on a node through
// offsets that differ in x or y: the z-column of one (c, ix, iy) offset is read, added and
// written as a batch; a compiler barrier keeps the next column's reads behind this
// column's writes (LDS executes a wave's instructions in order).
template <int O, int DIM, int CB, int CE>
__device__ __forceinline__ void cv_flush(const SubWin<O, DIM>& sw, const int* cc,
                                         const float* acc, float* win, bool own) {
  constexpr int A0 = acc_off<O, DIM>(CB);
#pragma unroll
  for (int c = CB; c < CE; ++c) {
    const int WX = cwin<O, DIM>(c, 0), WY = cwin<O, DIM>(c, 1), WZ = cwin<O, DIM>(c, 2);
    const int lx = cc[0] + win_lo(O, c == 0);
    const int ly = DIM >= 2 ? cc[1] + win_lo(O, c == 1) : 0;
    const int lz = DIM == 3 ? cc[2] + win_lo(O, c == 2) : 0;
    const int base = acc_off<O, DIM>(c) - A0;
#pragma unroll
    for (int iy = 0; iy < WY; ++iy)
#pragma unroll
      for (int ix = 0; ix < WX; ++ix) {
        if (own) {
          float v[5];
#pragma unroll
          for (int iz = 0; iz < WZ; ++iz) v[iz] = win[sw.index(c, lx + ix, ly + iy, lz + iz)];
#pragma unroll
          for (int iz = 0; iz < WZ; ++iz)
            win[sw.index(c, lx + ix, ly + iy, lz + iz)] =
                v[iz] + acc[base + (iz * WY + iy) * WX + ix];
        }
        asm volatile("" ::: "memory");
      }
  }
}

// One pass (components [CB, CE)) over a group, in rounds of CV_CAP staged slots.
template <int O, int DIM, int CB, int CE, bool LAST>
__device__ __forceinline__ void cv_pass(const KGrid& G, const KBins& B, const KPart& P,
                                        const TileBox& tb, const SubWin<O, DIM>& sw,
                                        const int32_t* s_off, const int32_t* s_len,
                                        const CellCtx& cx, CellStage& st, MoverBuf& mb,
                                        float* win, float* const* J, unsigned flags, double dt,
                                        uint32_t& bad) {
  constexpr int NA = acc_off<O, DIM>(CE) - acc_off<O, DIM>(CB);
  const int lane = cx.lane;
  const bool own = lane < cx.gn;
  const int cell = cx.g0 + (own ? lane : 0);
  int cc[3];
  {
    const int ex = tb.e[0], exy = tb.e[0] * tb.e[1];
    cc[2] = cell / exy;
    cc[1] = (cell - cc[2] * exy) / ex;
    cc[0] = cell - cc[2] * exy - cc[1] * ex;
#pragma unroll
    for (int d = 0; d < 3; ++d) cc[d] += tb.c0[d];
  }
  float acc[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) acc[i] = 0.0f;
  const int S0 = s_off[cx.g0], S1 = s_off[cx.g0 + cx.gn];
  for (int lo = S0; lo < S1; lo += CV_CAP) {
    const int hi = min(S1, lo + CV_CAP);
    cv_stage<O, DIM, LAST>(G, B, P, tb, s_off, s_len, cx, lo, hi, st, mb, J, flags, dt, bad);
    cv_accumulate<O, DIM, CB, CE>(s_off, s_len, cell, own, lo, hi, st, acc);
    wave_sync_lds();
  }
  cv_flush<O, DIM, CB, CE>(sw, cc, acc, win, own && s_len[cell] > 0);
}

// LDS layout of one workgroup (bytes).
template <int O, int DIM>
struct CellLayout {
  size_t sub_off, stage_off, total;
  int sub_floats;
  __host__ __device__ explicit CellLayout(const KBins& kb) {
    sub_floats = 3 * SubWin<O, DIM>::max_size(kb, CV_WAVES);
    sub_off = tile_smem_head(kb);
    stage_off = (sub_off + (size_t)CV_WAVES * sub_floats * sizeof(float) + 15) & ~(size_t)15;
    total = stage_off + (size_t)CV_WAVES * sizeof(CellStage);
  }
};

template <int O, int DIM>
__global__ __launch_bounds__(CV_WAVES * PIC_WAVE) void k_dep_cell_valu(
    KGrid G, KBins B, KPart P, float* __restrict__ J0, float* __restrict__ J1,
    float* __restrict__ J2, unsigned flags, double dt) {
  constexpr int SD = DIM - 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const CellLayout<O, DIM> L(B);
  const TileBox tb = tile_box(G.n, B.T, B.nt, blockIdx.x);
  const TileWin<O, DIM> tw(tb);
  int32_t* s_off = (int32_t*)smem_raw;
  int32_t* s_len = s_off + tb.nb + 1;
  float* J[3] = {J0, J1, J2};
  const int wave = threadIdx.x / PIC_WAVE;
  const int lane = threadIdx.x % PIC_WAVE;
  const int ns = tb.e[SD];
  const int slab = (ns + CV_WAVES - 1) / CV_WAVES;
  const int s0 = min(ns, wave * slab), s1 = min(ns, s0 + slab);
  const SubWin<O, DIM> sw(tw, s0, s1);
  float* win = (float*)(smem_raw + L.sub_off) + wave * L.sub_floats;
  CellStage& st = ((CellStage*)(smem_raw + L.stage_off))[wave];
  MoverBuf mb{st.mslot, st.mold, st.mnew, 0};
  for (int i = threadIdx.x; i <= tb.nb; i += blockDim.x) s_off[i] = B.off[tb.b0 + i];
  for (int i = threadIdx.x; i < tb.nb; i += blockDim.x) s_len[i] = B.len[tb.b0 + i];
  for (int i = lane; i < 3 * sw.size; i += PIC_WAVE) win[i] = 0.0f;
  __syncthreads();
  uint32_t bad = 0;
  // groups of the slab: 3D one z-plane chunk at a time; 2D chunks of the slab's rows
  const int ex = tb.e[0], exy = tb.e[0] * tb.e[1];
  const int plane = DIM == 3 ? exy : ex;          // cells per slab plane
  const int per_plane = (plane + CV_GROUP - 1) / CV_GROUP;
  for (int gi = 0; gi < (s1 - s0) * per_plane; ++gi) {
    const int pz = s0 + gi / per_plane;
    CellCtx cx;
    cx.lane = lane;
    cx.g0 = pz * plane + (gi % per_plane) * CV_GROUP;
    cx.gn = min(CV_GROUP, (pz + 1) * plane - cx.g0);
    if constexpr (O == 3 && DIM == 3) {
      cv_pass<O, DIM, 0, 2, false>(G, B, P, tb, sw, s_off, s_len, cx, st, mb, win, J, flags, dt, bad);
      cv_pass<O, DIM, 2, 3, true>(G, B, P, tb, sw, s_off, s_len, cx, st, mb, win, J, flags, dt, bad);
    } else {
      cv_pass<O, DIM, 0, 3, true>(G, B, P, tb, sw, s_off, s_len, cx, st, mb, win, J, flags, dt, bad);
    }
  }
  if (flags & PIC_F_EMIT_MOVERS) mb_flush(mb, B);
  if (bad) atomicOr(B.err, bad);
  __syncthreads();
  // tile window = sum of the slab sub-windows (overlapping along SD), to the scratch slab
  float* dst = B.wscr + (int64_t)blockIdx.x * 3 * B.wmax;
  const float* sub0 = (const float*)(smem_raw + L.sub_off);
  for (int i = threadIdx.x; i < 3 * tw.size; i += blockDim.x) {
    const int c = i / tw.size;
    const int r = i - c * tw.size;
    const int W01 = tw.W[0] * tw.W[1];
    const int z = r / W01, y = (r - z * W01) / tw.W[0], x = r - z * W01 - y * tw.W[0];
    const int sv = SD == 2 ? z : y;               // index along the slab dimension
    float v = 0.0f;
    for (int w = 0; w < CV_WAVES; ++w) {
      const int a0 = min(ns, w * slab), a1 = min(ns, a0 + slab);
      if (a1 <= a0) continue;
      const int ws = (a1 - a0) + TileWin<O, DIM>::R;
      const int q = sv - a0;
      if (q < 0 || q >= ws) continue;
      const int Wsub0 = tw.W[0];
      const int Wsub1 = SD == 1 ? ws : tw.W[1];
      const int Wsub2 = SD == 2 ? ws : tw.W[2];
      const int zz = SD == 2 ? q : z, yy = SD == 1 ? q : y;
      v += sub0[w * L.sub_floats + c * (Wsub0 * Wsub1 * Wsub2) + (zz * Wsub1 + yy) * Wsub0 + x];
    }
    dst[(int64_t)c * B.wmax + r] = v;
  }
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
