// Per-cell deposition on VALU: the rhocell of Sec. 3.4 (Eq. 4) / Sec. 4.2.1 kept in
// registers.
//
// One wave owns one particle tile and walks it in groups of up to 64 consecutive cells of
// one z-plane of the tile (bins are contiguous, so a group's particles are one
// contiguous slot range).
//  stage      lanes = slots, coalesced loads: position -> cell + float32 offset (FP64
//             only here), amplitude q W v_c, validity; the fused drift and mover
//             detection (stage 1 of Alg. 2) also run here, once per particle. Offsets and
//             amplitudes go to LDS. A particle whose cell no longer matches its bin is
//             deposited right away through the per-particle path (exact, rare).
//  accumulate lanes = cells: each lane walks its cell's staged particles and accumulates
//             the separable outer product (amp_c s_x) (x) s_y (x) s_z on the cell's padded
//             stencil window in registers (Eq. 4).
//  flush      once per cell, into the tile's LDS window (Eq. 5). Within one instruction
//             every lane adds at the same offset from its own cell, so the 64 addresses
//             differ and a plain read-add-write is race free; LDS float atomics, which
//             cost about 190 LDS cycles per wave instruction on this part, are not used.
//             The tile window is stored once and k_halo_sum adds neighbouring windows.
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

constexpr int CV_GROUP = 64;    // cells per wave group
constexpr int CV_CAP = 512;     // staged slots per wave per round
constexpr int CV_WAVES = 1;

// Per-wave staging area (SoA): offsets and amplitudes of CV_CAP slots.
struct Stage {
  float f[3][CV_CAP];
  float a[3][CV_CAP];
};

// Stage slots [lo, hi) of a cell group: lanes = slots.
template <int O, int DIM, bool LAST>
__device__ __forceinline__ void cv_stage(const KGrid& G, const KBins& B, const KPart& P,
                                         const TileBox& tb, const TileWin<O, DIM>& tw,
                                         const int32_t* s_off, const int32_t* s_len, int g0,
                                         int gn, int lo, int hi, Stage& st, float* win,
                                         float* const* J, unsigned flags, double dt,
                                         uint32_t& bad) {
  const int lane = __lane_id();
  const bool emit = LAST && (flags & PIC_F_EMIT_MOVERS);
  const bool drift = LAST && (flags & PIC_F_DRIFT);
  const int ex = tb.e[0], exy = tb.e[0] * tb.e[1];
  for (int base = lo; base < hi; base += PIC_WAVE) {
    const int s = base + lane;
    bool act = s < hi;
    int lb = 0;
    if (act) {
      int l = 0, h = gn;  // bin of slot s inside the group (s_off[g0 .. g0 + gn])
      while (h - l > 1) {
        int m = (l + h) >> 1;
        if (s_off[g0 + m] <= s) l = m;
        else h = m;
      }
      lb = g0 + l;
      act = s < s_off[lb] + s_len[lb];
    }
    PartPrep<O, DIM> p;
    double pos[3] = {0.0, 0.0, 0.0};
    float ux = 0.f, uy = 0.f, uz = 0.f;
    bool ok = false;
    if (act) {
      pos[0] = P.x[s];
      pos[1] = P.y[s];
      if (DIM == 3) pos[2] = P.z[s];
      ok = prep_cell<DIM>(G, pos[0], pos[1], pos[2], p.cell, p.f, bad);
    }
    bool mine = false;
    if (ok) {
      ux = P.ux[s];
      uy = P.uy[s];
      uz = P.uz[s];
      prep_amp(G.q, ux, uy, uz, P.w[s], p.amp);
      int cz = lb / exy, cy = (lb - cz * exy) / ex, cx = lb - cz * exy - cy * ex;
      mine = p.cell[0] == tb.c0[0] + cx && p.cell[1] == tb.c0[1] + cy &&
             (DIM == 2 || p.cell[2] == tb.c0[2] + cz);
      if (!mine && LAST) {
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
    }
    if (s < hi) {
      const int k = s - lo;
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
      int e = wave_append(mv, &B.ctr[CTR_NMOV]);
      if (mv) {
        if (e < B.max_movers) {
          B.mv_slot[e] = s;
          B.mv_old[e] = tb.b0 + lb;
          B.mv_new[e] = nbn;
        } else {
          atomicAdd(&B.ctr[CTR_NDROP], 1);
        }
      }
    }
  }
}

// Accumulate components [CB, CE) of the group's cells from the staged slots [lo, hi).
template <int O, int DIM, int CB, int CE, int NA>
__device__ __forceinline__ void cv_accumulate(const int32_t* s_off, const int32_t* s_len,
                                              int cell, bool own, int lo, int hi,
                                              const Stage& st, float* acc) {
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
    // 1D factors of the components in this pass, placed on the padded windows
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
  (void)NA;
}

// Add the cell's accumulators to the tile window with plain read-add-write. All cells of
// a group lie in one z-plane of the tile, so two lanes can only meet on a window node
// through offsets that differ in x or y: the z-column of one (c, ix, iy) offset is read,
// added and written as a batch, and a compiler barrier keeps the next column's reads
// behind this column's writes (LDS executes a wave's instructions in order).
template <int O, int DIM, int CB, int CE>
__device__ __forceinline__ void cv_flush(const TileWin<O, DIM>& tw, const int* cc,
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
          for (int iz = 0; iz < WZ; ++iz) v[iz] = win[tw.index(c, lx + ix, ly + iy, lz + iz)];
#pragma unroll
          for (int iz = 0; iz < WZ; ++iz)
            win[tw.index(c, lx + ix, ly + iy, lz + iz)] =
                v[iz] + acc[base + (iz * WY + iy) * WX + ix];
        }
        asm volatile("" ::: "memory");
      }
  }
}

// One pass (components [CB, CE)) over a cell group, in rounds of CV_CAP staged slots.
template <int O, int DIM, int CB, int CE, bool LAST>
__device__ __forceinline__ void cv_pass(const KGrid& G, const KBins& B, const KPart& P,
                                        const TileBox& tb, const TileWin<O, DIM>& tw,
                                        const int32_t* s_off, const int32_t* s_len, int g0,
                                        int gn, Stage& st, float* win, float* const* J,
                                        unsigned flags, double dt, uint32_t& bad) {
  constexpr int NA = acc_off<O, DIM>(CE) - acc_off<O, DIM>(CB);
  const int lane = __lane_id();
  const bool own = lane < gn;
  const int cell = g0 + (own ? lane : 0);
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
  const int S0 = s_off[g0], S1 = s_off[g0 + gn];
  for (int lo = S0; lo < S1; lo += CV_CAP) {
    const int hi = min(S1, lo + CV_CAP);
    cv_stage<O, DIM, LAST>(G, B, P, tb, tw, s_off, s_len, g0, gn, lo, hi, st, win, J, flags, dt,
                           bad);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    cv_accumulate<O, DIM, CB, CE, NA>(s_off, s_len, cell, own, lo, hi, st, acc);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  cv_flush<O, DIM, CB, CE>(tw, cc, acc, win, own && s_len[cell] > 0);
}

template <int O, int DIM>
__global__ __launch_bounds__(CV_WAVES * PIC_WAVE) void k_dep_cell_valu(
    KGrid G, KBins B, KPart P, float* __restrict__ J0, float* __restrict__ J1,
    float* __restrict__ J2, unsigned flags, double dt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileBox tb = tile_box(G.n, B.T, B.nt, blockIdx.x);
  const TileWin<O, DIM> tw(tb);
  int32_t* s_off = (int32_t*)smem_raw;
  int32_t* s_len = s_off + tb.nb + 1;
  float* win = (float*)(smem_raw + tile_smem_head(B));
  Stage* stage = (Stage*)(win + 3 * TileWin<O, DIM>::max_size(B));
  float* J[3] = {J0, J1, J2};
  for (int i = threadIdx.x; i <= tb.nb; i += blockDim.x) s_off[i] = B.off[tb.b0 + i];
  for (int i = threadIdx.x; i < tb.nb; i += blockDim.x) s_len[i] = B.len[tb.b0 + i];
  for (int i = threadIdx.x; i < 3 * tw.size; i += blockDim.x) win[i] = 0.0f;
  __syncthreads();
  uint32_t bad = 0;
  const int wave = threadIdx.x / PIC_WAVE;
  Stage& st = stage[wave];
  const int exy = tb.e[0] * tb.e[1];
  const int per_plane = (exy + CV_GROUP - 1) / CV_GROUP;
  for (int gi = wave; gi < per_plane * tb.e[2]; gi += CV_WAVES) {
    const int pz = gi / per_plane;
    const int g0 = pz * exy + (gi - pz * per_plane) * CV_GROUP;
    const int gn = min(CV_GROUP, (pz + 1) * exy - g0);
    if constexpr (O == 3 && DIM == 3) {
      cv_pass<O, DIM, 0, 2, false>(G, B, P, tb, tw, s_off, s_len, g0, gn, st, win, J, flags, dt, bad);
      cv_pass<O, DIM, 2, 3, true>(G, B, P, tb, tw, s_off, s_len, g0, gn, st, win, J, flags, dt, bad);
    } else {
      cv_pass<O, DIM, 0, 3, true>(G, B, P, tb, tw, s_off, s_len, g0, gn, st, win, J, flags, dt, bad);
    }
  }
  if (bad) atomicOr(B.err, bad);
  __syncthreads();
  store_window<O, DIM>(B, blockIdx.x, tw, win, blockDim.x, threadIdx.x);
}

// ---------------------------------------------------------------------------------
bool deposit_mfma_launch(const KGrid& G, const KPart& P, pic_bins* b, float* J0, float* J1,
                         float* J2, int path, unsigned flags, double dt, hipStream_t s);

template <int O, int DIM>
static bool launch_cell_valu(const KGrid& G, const KPart& P, pic_bins* b, float* J0, float* J1,
                             float* J2, unsigned flags, double dt, hipStream_t s) {
  size_t smem = tile_smem_head(b->kb) + 3 * sizeof(float) * TileWin<O, DIM>::max_size(b->kb) +
                CV_WAVES * sizeof(Stage);
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
