// Per-cell deposition on VALU: the rhocell of Sec. 3.4 (Eq. 4) / Sec. 4.2.1 kept in
// registers.
//
// A workgroup owns one particle tile and walks it in groups of 64 consecutive cells (one
// z-plane of an 8 x 8 x T tile). A unit takes up to k particles of every cell of a group
// (at most 512 in all; a group that fits is one unit, a dense one is cut across its cells),
// so every cell lane has work at any density. Four waves:
//  producer   (wave 3) stages unit u + 1 while the consumers work on unit u. Lanes = the
//             unit's particles (each one's cell read from the unit's table, built by the
//             cell lanes, so gap slots take no lane), coalesced loads: position -> cell
//             + float32 offset (FP64 only here) and amplitude q W v_c. Offsets and
//             amplitudes go to a double-buffered LDS stage in cell order. A particle whose
//             cell no longer matches its bin goes to a stale list.
//  consumers  (wave c = 0, 1, 2: component c) lanes = cells: each lane walks its cell's
//             staged particles and accumulates (amp_c s_x) (x) s_y (x) s_z of component c
//             on the cell's padded stencil window in registers (Eq. 4); after the group's
//             last unit it adds them to the tile window in LDS (Eq. 5) with plain
//             read-add-write. After each unit they and the producer (after staging the
//             next unit) share the fused drift and mover detection (stage 1 of Alg. 2) of
//             its particles, a quarter each, movers going to per-wave LDS buffers. The
//             consumers write different components, so they never share a word. LDS float atomics cost about 190 cycles per wave instruction
//             on gfx950 (integer ones about 5) and are not used.
//  end        the consumers add the stale particles (one at a time, lanes = stencil nodes)
//             and the tile window goes to the window scratch; k_halo_tile adds neighbouring
//             tiles into J.
// Staggered axes use a window one node wider than the stencil (the stencil of a particle
// in cell i starts at i + lo or i + lo + 1 depending on which half of the cell it is in);
// the extra node carries a zero weight.
#include "deposit_common.h"

// Window extent of accumulator set c along d: component c of J is staggered along its own
// axis; the charge density (RHO) is nodal everywhere.
template <int O, int DIM, bool RHO = false>
__host__ __device__ constexpr int cwin(int c, int d) {
  return d < DIM ? win_w(O, !RHO && c == d) : 1;
}
template <int O, int DIM, bool RHO = false>
__host__ __device__ constexpr int csz(int c) {
  return cwin<O, DIM, RHO>(c, 0) * cwin<O, DIM, RHO>(c, 1) * cwin<O, DIM, RHO>(c, 2);
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

// Inclusive scan of v over the wave's 64 lanes with DPP moves: shifts by 1, 2, 4 and 8
// lanes inside each 16-lane row, then lane 15 of rows 0 and 2 added into rows 1 and 3 and
// lane 31 into rows 2 and 3. VALU only (a lane shuffle is an LDS round trip); all 64 lanes
// must be active. `id` is the identity of `op`.
struct DppAdd {
  __device__ int operator()(int a, int b) const { return a + b; }
};
struct DppMax {
  __device__ int operator()(int a, int b) const { return a > b ? a : b; }
};
template <typename Op>
__device__ __forceinline__ int wave_scan(int v, int id, Op op) {
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x111, 0xf, 0xf, false));   // row_shr:1
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x112, 0xf, 0xf, false));   // row_shr:2
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x114, 0xf, 0xf, false));   // row_shr:4
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x118, 0xf, 0xf, false));   // row_shr:8
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x142, 0xa, 0xf, false));   // row_bcast:15
  v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x143, 0xc, 0xf, false));   // row_bcast:31
  return v;
}

// Wave-uniform maximum of a non-negative v.
__device__ __forceinline__ int wave_max(int v) {
  return __builtin_amdgcn_readlane(wave_scan(v, 0, DppMax()), PIC_WAVE - 1);
}

constexpr int CV_GROUP = 64;    // cells per group (lanes)
constexpr int CV_CAP = 512;     // staged particles per unit (gap slots skipped)
// Per-unit table (bytes): the cell (group lane) of each staged particle, int8[CV_CAP], with
// CV_TAB_BAD set when the producer found its position outside the domain or not finite,
// then each cell's staged start minus its particles staged by earlier units of the group,
// int32[CV_GROUP] (staged index + that = index inside the cell's bin); double-buffered like
// the stage.
constexpr int CV_TAB = CV_CAP + 4 * CV_GROUP;
constexpr int CV_TAB_BAD = 64;   // table flag: the particle's staged position is not valid
constexpr int CV_CONS = 3;      // consumer waves, one per current component
constexpr int CV_PROD = 1;      // producer waves
constexpr int CV_WAVES = CV_CONS + CV_PROD;
constexpr int CV_STALE = 128;   // stale particles a tile keeps for the end phase
// Staged amplitudes carry 1/6^DIM at third order: the consumers use weights times 6.
template <int O, int DIM>
constexpr float CV_AMP_SCALE = O == 3 ? (DIM == 3 ? 1.0f / 216.0f : 1.0f / 36.0f) : 1.0f;

// Position of staged particle q in a stage array. The consumers read one particle per
// lane at q = (cell start) + k, so with a uniform count of n particles per cell the lanes'
// addresses are n words apart, and n = 8 would put every fourth lane in one LDS bank.
// Flipping the low three bits of q with bits 5-7 (a permutation of each 256-word block)
// spreads such strides over all banks; consecutive q stay conflict-free for the producer.
__device__ __forceinline__ int cv_sw(int q) { return q ^ ((q >> 5) & 7); }

// A particle found in the bin of another cell, kept for the end phase.
struct StaleRec {
  int cell[3];
  float f[3];
  float amp[3];
};

// LDS layout of one workgroup (bytes): bin offsets and lengths | tile window (3 comps)
// | two stage buffers f[3][CAP], a[3][CAP] | two unit tables | per wave: mover buffer
// | stale list and its count.
template <int O, int DIM>
struct CellLayout {
  size_t win_off, stage_off, tab_off, mb_off, stale_off, total;
  __host__ __device__ explicit CellLayout(const KBins& kb) {
    win_off = tile_smem_head(kb);
    stage_off = win_off + (((size_t)3 * TileWin<O, DIM>::max_size(kb) * sizeof(float) + 15) & ~(size_t)15);
    tab_off = stage_off + (size_t)2 * 6 * CV_CAP * sizeof(float);
    mb_off = tab_off + (size_t)2 * CV_TAB;
    stale_off = mb_off + (size_t)CV_WAVES * 3 * MBUF * sizeof(int32_t);
    total = stale_off + (size_t)CV_STALE * sizeof(StaleRec) + 16;
  }
};

// A unit of work: up to k particles of every cell of one group of 64 consecutive cells, the
// next ones of each cell (in slot order) after those of the group's earlier units, with k
// the largest count that keeps the unit within CV_CAP particles. A group that fits takes one
// unit; a dense group is cut across its cells (k >= CV_CAP / 64), so the 64 consumer lanes
// (one per cell) all have particles whatever the density. Every wave walks the same
// sequence of units (empty groups skipped).
struct CellGroup {
  int g0, gn;        // first tile-local bin, cells
  int n;             // this lane's cell: particles (valid slots)
  int done;          // this lane's cell: particles staged by the group's earlier units
  int m, ust;        // this lane's cell in this unit: particles, staged start
  int nunit;         // particles of this unit
  bool last;         // no particles of the group are left after this unit
};

__device__ __forceinline__ int wave_sum(int v) {
  return __builtin_amdgcn_readlane(wave_scan(v, 0, DppAdd()), PIC_WAVE - 1);
}

// Per-lane count and staged start of the next unit of the group (wave reductions and a scan
// over the group's cells).
__device__ __forceinline__ void cv_unit_fields(CellGroup& gr, int lane) {
  const int r = gr.n - gr.done;
  const int rtot = wave_sum(r);
  int k = wave_max(r);
  if (rtot > CV_CAP) {
    // largest k with sum_c min(r_c, k) <= CV_CAP (k = 1 always fits: 64 <= CV_CAP)
    int lo = 1, hi = k;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (wave_sum(min(r, mid)) <= CV_CAP) lo = mid;
      else hi = mid - 1;
    }
    k = lo;
  }
  const int m = min(r, k);
  const int incl = wave_scan(m, 0, DppAdd());
  gr.m = m;
  gr.ust = incl - m;
  gr.nunit = __builtin_amdgcn_readlane(incl, PIC_WAVE - 1);
  gr.last = gr.nunit == rtot;
}

// The group starting at tile-local bin g0 (g0 >= nb: past the end, no particles), at its
// first unit. Every field is written once per unit, so the struct stays in registers.
__device__ __forceinline__ CellGroup cv_group_at(int g0, const int32_t* s_off,
                                                 const int32_t* s_len, int nb, int lane) {
  const bool valid = g0 < nb;
  const int gs = valid ? g0 : 0;
  const int gn = valid ? min(CV_GROUP, nb - g0) : 0;
  CellGroup gr;
  gr.g0 = g0;
  gr.gn = gn;
  gr.n = lane < gn ? s_len[gs + lane] : 0;
  gr.done = 0;
  cv_unit_fields(gr, lane);
  return gr;
}

__device__ __forceinline__ CellGroup cv_first_unit(int g0, const int32_t* s_off,
                                                   const int32_t* s_len, int nb, int lane) {
  CellGroup gr = cv_group_at(g0, s_off, s_len, nb, lane);
  while (gr.g0 < nb && gr.nunit == 0) gr = cv_group_at(gr.g0 + CV_GROUP, s_off, s_len, nb, lane);
  return gr;
}

__device__ __forceinline__ CellGroup cv_next_unit(const CellGroup& cur, const int32_t* s_off,
                                                  const int32_t* s_len, int nb, int lane) {
  if (!cur.last) {
    CellGroup gr = cur;
    gr.done = cur.done + cur.m;
    cv_unit_fields(gr, lane);
    return gr;
  }
  return cv_first_unit(cur.g0 + CV_GROUP, s_off, s_len, nb, lane);
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Raw particle data of one slot, fetched one chunk ahead of its use.
struct CvRaw {
  double x, y, z;
  float ux, uy, uz, w;
  int s, lc, si;
};

// One particle's charge density through global atomics (the rare overflow of a tile's
// stale list in the density mode).
template <int O, int DIM>
__device__ __forceinline__ void cv_rho_particle_global(const KGrid& G, const PartPrep<O, DIM>& p,
                                                       float* rho, uint32_t& bad) {
  float w[3][O + 1];
  int base[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d < DIM) {
      base[d] = p.cell[d] + win_lo(O, false) + shape_w<O, false>(p.f[d], w[d]);
    } else {
#pragma unroll
      for (int k = 0; k <= O; ++k) w[d][k] = k == 0 ? 1.0f : 0.0f;
    }
  }
  for (int kz = 0; kz < (DIM == 3 ? O + 1 : 1); ++kz)
    for (int ky = 0; ky <= O; ++ky)
      for (int kx = 0; kx <= O; ++kx) {
        const float v = p.amp[0] * w[0][kx] * w[1][ky] * w[2][kz];
        const int ix = store_idx(G, 0, base[0] + kx), iy = store_idx(G, 1, base[1] + ky);
        const int iz = DIM == 3 ? store_idx(G, 2, base[2] + kz) : 0;
        if ((ix | iy | iz) < 0) {
          if (v != 0.0f) bad |= PIC_EF_STENCIL;
          continue;
        }
        unsafeAtomicAdd(&rho[((int64_t)iz * G.N[1] + iy) * G.N[0] + ix], v);
      }
}

// w[i] by selects (the empty asm keeps the compiler from turning it into an indexed
// load from a stack copy of w).
template <int O>
__device__ __forceinline__ float pick_w(const float* w, int i) {
  float v = w[0];
#pragma unroll
  for (int k = 1; k <= O; ++k) {
    float wk = w[k];
    asm volatile("" : "+v"(wk));
    v = i == k ? wk : v;
  }
  return v;
}

// One particle through global atomics (the rare overflow of a tile's stale list).
template <int O, int DIM>
__device__ __forceinline__ void cv_particle_global(const KGrid& G, PartPrep<O, DIM> p,
                                                float* const* J, uint32_t& bad) {
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

// Producer wave: stage the unit's particles (cell by cell, staged index in [0, nunit)) into
// one stage buffer, lanes = particles, so no lane idles on a gap slot. The unit's table gives
// each staged particle's cell (each cell lane writes its own range [st, st + n) of it) and
// each cell's staged start; the consumers' drift reads the same table. Coalesced loads;
// three chunks' loads are in flight ahead of the one being processed (memory latency,
// not the VALU, bounds this wave).
template <int O, int DIM, bool RHO>
__device__ __forceinline__ void cv_stage(const KGrid& G, const KBins& B, const KPart& P,
                                         const TileBox& tb, const int32_t* s_off,
                                         const int32_t* s_len, const CellGroup& gr, float* sf,
                                         float* sa, int8_t* tab, StaleRec* stale, int* s_nstale,
                                         float* const* J, uint32_t& bad, float hdt) {
  const int lane = threadIdx.x % PIC_WAVE;
  const int pw = threadIdx.x / PIC_WAVE - CV_CONS;   // producer index
  const int ex = tb.e[0];
  const int nunit = gr.nunit;
  const int first = pw * PIC_WAVE, step = CV_PROD * PIC_WAVE;
  int32_t* tst = (int32_t*)(tab + CV_CAP);
  wave_lds_sync();
  tst[lane] = gr.ust - gr.done;
  for (int k = 0; k < gr.m; ++k) tab[gr.ust + k] = (int8_t)lane;
  wave_lds_sync();
  auto fetch = [&](int base, CvRaw& r) {
    r.si = base + lane;
    r.lc = r.si < nunit ? (int)tab[r.si] : -1;
    r.s = r.lc >= 0 ? s_off[gr.g0 + r.lc] + (r.si - tst[r.lc]) : 0;
    if (r.lc >= 0) {
      r.x = P.x[r.s];
      r.y = P.y[r.s];
      r.z = DIM == 3 ? P.z[r.s] : 0.0;
      r.ux = P.ux[r.s];
      r.uy = P.uy[r.s];
      r.uz = P.uz[r.s];
      r.w = P.w[r.s];
    }
  };
  CvRaw nx1, nx2, nx3;
  if (first < nunit) fetch(first, nx1);
  if (first + step < nunit) fetch(first + step, nx2);
  if (first + 2 * step < nunit) fetch(first + 2 * step, nx3);
  for (int base = first; base < nunit; base += step) {
    const CvRaw r = nx1;
    nx1 = nx2;
    nx2 = nx3;
    if (base + 3 * step < nunit) fetch(base + 3 * step, nx3);
    const int lb = gr.g0 + (r.lc < 0 ? 0 : r.lc);
    PartPrep<O, DIM> p;
    double pos[3] = {r.x, r.y, r.z};
    bool ok = false, mine = false;
    if (r.lc >= 0) {
      // time-centred deposition at x + hdt v (hdt = +-dt/2)
      if (hdt != 0.0f) midpoint_shift<DIM>(G, pos, r.ux, r.uy, r.uz, hdt);
      ok = prep_cell<DIM>(G, pos[0], pos[1], pos[2], p.cell, p.f, bad);
      if (!ok) tab[r.si] = (int8_t)(r.lc | CV_TAB_BAD);   // the drift skips it
      if constexpr (RHO) {
        p.amp[0] = G.q * r.w;       // charge density: q W, no velocity
        p.amp[1] = p.amp[2] = 0.0f;
      } else {
        prep_amp_rsq(G.q, r.ux, r.uy, r.uz, r.w, 1.0f, p.amp);
      }
      // the particle's cell relative to the tile -> local bin (no division)
      const int lx = p.cell[0] - tb.c0[0], ly = p.cell[1] - tb.c0[1];
      const int lz = DIM == 3 ? p.cell[2] - tb.c0[2] : 0;
      const bool in = (unsigned)lx < (unsigned)tb.e[0] && (unsigned)ly < (unsigned)tb.e[1] &&
                      (unsigned)lz < (unsigned)(DIM == 3 ? tb.e[2] : 1);
      mine = ok && in && lx + ex * (ly + tb.e[1] * lz) == lb;
    }
    // stale particle (its cell no longer matches its bin): kept for the end phase, or,
    // when the tile's list is full, deposited at once through global atomics
    const bool st = ok && !mine;
    const unsigned long long m = __ballot(st);
    if (m) {
      int e0 = 0;
      if (lane == 0) e0 = atomicAdd(s_nstale, (int)__popcll(m));
      e0 = __shfl(e0, 0);
      const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
      if (st) {
        if (e0 + rank < CV_STALE) {
          StaleRec& q = stale[e0 + rank];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            q.cell[d] = d < DIM ? p.cell[d] : 0;
            q.f[d] = d < DIM ? p.f[d] : 0.0f;
            q.amp[d] = p.amp[d];
          }
        } else if constexpr (RHO) {
          cv_rho_particle_global<O, DIM>(G, p, J[0], bad);
        } else {
          cv_particle_global<O, DIM>(G, p, J, bad);
        }
      }
    }
    if (r.lc >= 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        sf[d * CV_CAP + cv_sw(r.si)] = mine ? p.f[d] : 0.0f;
        sa[d * CV_CAP + cv_sw(r.si)] = mine ? p.amp[d] * CV_AMP_SCALE<O, DIM> : 0.0f;
      }
    }
  }
}

// Shape weights as the consumers use them (third order: times 6, see CV_AMP_SCALE). In 2D
// the z weight is the constant 1 and is not scaled.
template <int O, bool STAG>
__device__ __forceinline__ int cv_shape(float f, float* w) {
  if constexpr (O == 3) return shape_w6<STAG>(f, w);
  else return shape_w<O, STAG>(f, w);
}

// Accumulate set C of the lane's cell from the staged particles [k0, k1): component C of J,
// or (RHO) every third particle starting at the C-th for the charge density, so the three
// waves share the particles of a cell and each fills its own copy of the window.
template <int O, int DIM, int C, bool RHO>
__device__ __forceinline__ void cv_accumulate(int k0, int k1, const float* sf, const float* sa,
                                              float* acc) {
  constexpr int WX = cwin<O, DIM, RHO>(C, 0), WY = cwin<O, DIM, RHO>(C, 1),
                WZ = cwin<O, DIM, RHO>(C, 2);
  constexpr int STEP = RHO ? 3 : 1;
  const int first = RHO ? k0 + C : k0;
  const int n = k1 > first ? (k1 - first + STEP - 1) / STEP : 0;
  const int nmax = wave_max(n);
  for (int k = 0; k < nmax; ++k) {
    const bool act = k < n;
    const int q = cv_sw(act ? first + k * STEP : 0);
    float f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) f[d] = sf[d * CV_CAP + q];
    const float amp = act ? sa[(RHO ? 0 : C) * CV_CAP + q] : 0.0f;
    float wx[5], wy[5], wz[5];
    {
      float w[O + 1];
      int sh = cv_shape<O, !RHO && C == 0>(f[0], w);
      pad_w<O, WX>(w, sh, wx);
      sh = cv_shape<O, !RHO && C == 1>(f[1], w);
      pad_w<O, WY>(w, sh, wy);
      if constexpr (DIM == 3) {
        sh = cv_shape<O, !RHO && C == 2>(f[2], w);
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
template <int O, int DIM, int C, bool ZBATCH, bool RHO>
__device__ __forceinline__ void cv_flush(const TileWin<O, DIM>& tw, const int* cc,
                                         const float* acc, float* win, bool own) {
  constexpr int WX = cwin<O, DIM, RHO>(C, 0), WY = cwin<O, DIM, RHO>(C, 1),
                WZ = cwin<O, DIM, RHO>(C, 2);
  const int lx = cc[0] + win_lo(O, !RHO && C == 0);
  const int ly = cc[1] + win_lo(O, !RHO && C == 1);
  const int lz = DIM == 3 ? cc[2] + win_lo(O, !RHO && C == 2) : 0;
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

template <int O, int DIM, bool RHO = false>
__host__ __device__ constexpr int csz_max() {
  return csz<O, DIM, RHO>(0) > csz<O, DIM, RHO>(1)
             ? (csz<O, DIM, RHO>(0) > csz<O, DIM, RHO>(2) ? csz<O, DIM, RHO>(0) : csz<O, DIM, RHO>(2))
             : (csz<O, DIM, RHO>(1) > csz<O, DIM, RHO>(2) ? csz<O, DIM, RHO>(1) : csz<O, DIM, RHO>(2));
}


// End phase, wave C: component C of every stale particle of the tile, one particle at a
// time with lanes = stencil nodes (distinct nodes, so plain read-add-write into the tile
// window; nodes outside the window go to J with global atomics).
template <int O, int DIM, int C, bool RHO>
__device__ __forceinline__ void cv_stale(const KGrid& G, const TileWin<O, DIM>& tw,
                                         const StaleRec* stale, int nstale, float* win,
                                         float* const* J, uint32_t& bad) {
  if constexpr (RHO && C != 0) return;      // the density has one set: wave 0 adds it
  constexpr int NS = (O + 1) * (O + 1) * (DIM == 3 ? O + 1 : 1);
  const int lane = threadIdx.x % PIC_WAVE;
  for (int e = 0; e < nstale; ++e) {
    const StaleRec q = stale[e];
    float w[3][O + 1];
    int base[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      int sh;
      if (!RHO && d == C) sh = shape_w<O, true>(q.f[d], w[d]);
      else sh = shape_w<O, false>(q.f[d], w[d]);
      base[d] = q.cell[d] + win_lo(O, !RHO && d == C) + sh;
    }
    for (int j = lane; j < NS; j += PIC_WAVE) {
      const int ix = j % (O + 1), iy = (j / (O + 1)) % (O + 1), iz = j / ((O + 1) * (O + 1));
      float v = q.amp[C] * pick_w<O>(w[0], ix) * pick_w<O>(w[1], iy);
      if (DIM == 3) v *= pick_w<O>(w[2], iz);
      const int m[3] = {base[0] + ix, base[1] + iy, DIM == 3 ? base[2] + iz : 0};
      bool in = true;
#pragma unroll
      for (int d = 0; d < DIM; ++d) in = in && m[d] >= tw.o[d] && m[d] < tw.o[d] + tw.W[d];
      if (in) {
        const int a = tw.index(C, m[0], m[1], m[2]);
        win[a] = win[a] + v;
      } else {
        const int sx = store_idx(G, 0, m[0]), sy = store_idx(G, 1, m[1]);
        const int sz = DIM == 3 ? store_idx(G, 2, m[2]) : 0;
        if ((sx | sy | sz) < 0) {
          if (v != 0.0f) bad |= PIC_EF_STENCIL;
        } else {
          unsafeAtomicAdd(&J[C][((int64_t)sz * G.N[1] + sy) * G.N[0] + sx], v);
        }
      }
    }
    asm volatile("" ::: "memory");
  }
}

// Consumer wave C: flush component C of the group's cells into the tile window.
template <int O, int DIM, int C, bool RHO>
__device__ __forceinline__ void cv_flush_group(const TileBox& tb, const TileWin<O, DIM>& tw,
                                               const CellGroup& gr, const float* acc,
                                               float* win) {
  const int lane = threadIdx.x % PIC_WAVE;
  const bool own = lane < gr.gn;
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
  if (plane) cv_flush<O, DIM, C, true, RHO>(tw, cc, acc, win, o);
  else cv_flush<O, DIM, C, false, RHO>(tw, cc, acc, win, o);
}

// Fused drift (x += v dt, FP64) and mover detection (stage 1 of Alg. 2) of a unit, lanes =
// particles (each one's cell and slot from the unit's table, so gap slots take no lane):
// wave w takes chunk j of 64 when j mod 4 = w. The three accumulating waves do theirs after
// accumulating the unit, the producer after staging the next unit: the accumulation keeps
// the consumers' SIMDs busier than the producer's, so the producer takes an equal share.
template <int DIM>
__device__ __forceinline__ void cv_drift_unit(const KGrid& G, const KBins& B, const KPart& P,
                                              const TileBox& tb, const int32_t* s_off,
                                              const int32_t* s_len, const CellGroup& gr,
                                              const int8_t* tab, bool tab_ok, int wave,
                                              MoverBuf& mb, unsigned flags, double dt,
                                              uint32_t& bad) {
  const int lane = threadIdx.x % PIC_WAVE;
  const bool emit = flags & PIC_F_EMIT_MOVERS;
  const bool drift = flags & PIC_F_DRIFT;
  const int ex = tb.e[0];
  const int nunit = gr.nunit;
  for (int base = wave * PIC_WAVE; base < nunit; base += CV_WAVES * PIC_WAVE) {
    const int j = base + lane;
    const bool in_unit = j < nunit;
    const int tv = in_unit ? (int)tab[j] : 0;
    const int c = tv & (CV_GROUP - 1);
    const int s = in_unit ? s_off[gr.g0 + c] + (j - ((const int32_t*)(tab + CV_CAP))[c]) : 0;
    const int lb = gr.g0 + (in_unit ? c : 0);
    bool ok = false, mv = false;
    int32_t nbn = -1;
    if (in_unit) {
      double pos[3] = {P.x[s], P.y[s], DIM == 3 ? P.z[s] : 0.0};
      int c1[3];
      float f1[3];
      uint32_t nb0 = 0;   // errors are reported by the producer
      // the producer checked this same position unless it staged a shifted one
      if (tab_ok) ok = !(tv & CV_TAB_BAD);
      else ok = prep_cell<DIM>(G, pos[0], pos[1], pos[2], c1, f1, nb0);
      if (ok && drift) {
        drift_one<DIM>(G, pos, P.ux[s], P.uy[s], P.uz[s], dt);
        P.x[s] = pos[0];
        P.y[s] = pos[1];
        if (DIM == 3) P.z[s] = pos[2];
      }
      if (ok && emit) {
        // mover: its (new) cell differs from the cell of the bin it sits in
        int c2[3];
        float f2[3];
        if (prep_cell<DIM>(G, pos[0], pos[1], pos[2], c2, f2, bad)) {
          const int lx = c2[0] - tb.c0[0], ly = c2[1] - tb.c0[1];
          const int lz = DIM == 3 ? c2[2] - tb.c0[2] : 0;
          const bool in = (unsigned)lx < (unsigned)tb.e[0] && (unsigned)ly < (unsigned)tb.e[1] &&
                          (unsigned)lz < (unsigned)(DIM == 3 ? tb.e[2] : 1);
          const int loc = lx + ex * (ly + tb.e[1] * lz);
          mv = !(in && loc == lb);
          if (mv) nbn = in ? tb.b0 + loc : bin_of_cell(G.n, B.T, c2[0], c2[1], c2[2]);
        }
      }
    }
    if (emit) mb_append(mb, B, mv, s, tb.b0 + lb, nbn);
  }
}

template <int O, int DIM, int C, bool RHO>
__device__ __forceinline__ void cv_consume(int k0, int k1, const float* sf, const float* sa,
                                           float* acc, bool last, const TileBox& tb,
                                           const TileWin<O, DIM>& tw, const CellGroup& gr,
                                           float* win) {
  cv_accumulate<O, DIM, C, RHO>(k0, k1, sf, sa, acc);
  if (last) {
    cv_flush_group<O, DIM, C, RHO>(tb, tw, gr, acc, win);
#pragma unroll
    for (int i = 0; i < csz_max<O, DIM, RHO>(); ++i) acc[i] = 0.0f;
  }
}

// One workgroup per tile: the producer wave(s) stage unit u + 1 while waves 0..2 accumulate
// unit u. Every wave walks the same units and passes the same number of barriers. (A
// workgroup of more than four waves was measured to fit only once per CU.)
template <int O, int DIM, bool RHO = false>
__device__ __forceinline__ void cell_tile(const KGrid& G, const KBins& B, const KPart& P,
                                          float* J0, float* J1, float* J2, unsigned flags,
                                          double dt, int tile, unsigned char* smem_raw) {
  constexpr int NA = csz_max<O, DIM, RHO>();
  const CellLayout<O, DIM> L(B);
  const TileBox tb = tile_box(G.n, B.T, B.nt, tile);
  const TileWin<O, DIM> tw(tb);
  int32_t* s_off = (int32_t*)smem_raw;
  int32_t* s_len = s_off + tb.nb + 1;
  float* win = (float*)(smem_raw + L.win_off);
  float* stage = (float*)(smem_raw + L.stage_off);
  int8_t* tab = (int8_t*)(smem_raw + L.tab_off);
  const int wave = threadIdx.x / PIC_WAVE;
  const int lane = threadIdx.x % PIC_WAVE;
  const bool producer = wave >= CV_CONS;
  int32_t* mbb = (int32_t*)(smem_raw + L.mb_off) + wave * 3 * MBUF;
  StaleRec* stale = (StaleRec*)(smem_raw + L.stale_off);
  int* s_nstale = (int*)(smem_raw + L.stale_off + CV_STALE * sizeof(StaleRec));
  float* J[3] = {J0, J1, J2};
  MoverBuf mb{mbb, mbb + MBUF, mbb + 2 * MBUF, 0};
  for (int i = threadIdx.x; i <= tb.nb; i += blockDim.x) s_off[i] = B.off[tb.b0 + i];
  for (int i = threadIdx.x; i < tb.nb; i += blockDim.x) s_len[i] = B.len[tb.b0 + i];
  for (int i = threadIdx.x; i < 3 * tw.size; i += blockDim.x) win[i] = 0.0f;
  if (threadIdx.x == 0) *s_nstale = 0;
  __syncthreads();
  uint32_t bad = 0;
  const float hdt = (RHO || !(flags & PIC_F_MIDPOINT)) ? 0.0f
                    : (float)((flags & PIC_F_DRIFT) ? 0.5 * dt : -0.5 * dt);
  CellGroup cur = cv_first_unit(0, s_off, s_len, tb.nb, lane);
  // The producer and the consumers run separate loops over the same units with one
  // barrier per unit (plus one after the first unit is staged), so the consumers'
  // accumulators are not live across the producer's code.
  const bool drift = !RHO && (flags & (PIC_F_DRIFT | PIC_F_EMIT_MOVERS));
  if (producer) {
    // Each SIMD runs waves of three workgroups, mostly consumers with long FMA streams; at
    // equal priority the producer, whose staging sets the pace of every unit, gets about a
    // third of the issue slots (measured: 7% faster deposition with the raise).
    __builtin_amdgcn_s_setprio(1);
    if (cur.g0 < tb.nb)
      cv_stage<O, DIM, RHO>(G, B, P, tb, s_off, s_len, cur, stage, stage + 3 * CV_CAP, tab,
                            stale, s_nstale, J, bad, hdt);
    __syncthreads();
    int ub = 0;
    while (cur.g0 < tb.nb) {
      const CellGroup nxt = cv_next_unit(cur, s_off, s_len, tb.nb, lane);
      if (nxt.g0 < tb.nb) {
        float* nf = stage + (ub ^ 1) * 6 * CV_CAP;
        cv_stage<O, DIM, RHO>(G, B, P, tb, s_off, s_len, nxt, nf, nf + 3 * CV_CAP,
                              tab + (ub ^ 1) * CV_TAB, stale, s_nstale, J, bad, hdt);
      }
      if (drift)
        cv_drift_unit<DIM>(G, B, P, tb, s_off, s_len, cur, tab + ub * CV_TAB, hdt == 0.0f, wave,
                           mb, flags, dt, bad);
      __syncthreads();
      cur = nxt;
      ub ^= 1;
    }
    if (!RHO && (flags & PIC_F_EMIT_MOVERS)) mb_flush(mb, B);
  } else {
    float acc[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) acc[i] = 0.0f;
    __syncthreads();
    int ub = 0;
    while (cur.g0 < tb.nb) {
      const CellGroup nxt = cv_next_unit(cur, s_off, s_len, tb.nb, lane);
      const float* sf = stage + ub * 6 * CV_CAP;
      const int k0 = cur.ust, k1 = cur.ust + cur.m;
      const bool last = cur.last;
      if (wave == 0) cv_consume<O, DIM, 0, RHO>(k0, k1, sf, sf + 3 * CV_CAP, acc, last, tb, tw, cur, win);
      else if (wave == 1) cv_consume<O, DIM, 1, RHO>(k0, k1, sf, sf + 3 * CV_CAP, acc, last, tb, tw, cur, win);
      else cv_consume<O, DIM, 2, RHO>(k0, k1, sf, sf + 3 * CV_CAP, acc, last, tb, tw, cur, win);
      // the drift share is on the unit's critical path like the producer's work
      __builtin_amdgcn_s_setprio(1);
      if (drift)
        cv_drift_unit<DIM>(G, B, P, tb, s_off, s_len, cur, tab + ub * CV_TAB, hdt == 0.0f, wave,
                           mb, flags, dt, bad);
      __syncthreads();
      __builtin_amdgcn_s_setprio(0);
      cur = nxt;
      ub ^= 1;
    }
    if (!RHO && (flags & PIC_F_EMIT_MOVERS)) mb_flush(mb, B);
  }
  __syncthreads();
  const int ns = min(*s_nstale, CV_STALE);
  if (ns > 0) {
    if (wave == 0) cv_stale<O, DIM, 0, RHO>(G, tw, stale, ns, win, J, bad);
    else if (wave == 1) cv_stale<O, DIM, 1, RHO>(G, tw, stale, ns, win, J, bad);
    else if (wave == 2) cv_stale<O, DIM, 2, RHO>(G, tw, stale, ns, win, J, bad);
  }
  if (bad) atomicOr(B.err, bad);
  __syncthreads();
  store_window(B, tile, tw, win, blockDim.x, threadIdx.x);
}

template <int O, int DIM>
__global__ __launch_bounds__(CV_WAVES * PIC_WAVE, 3) void k_dep_cell_valu(
    KGrid G, KBins B, KPart P, float* __restrict__ J0, float* __restrict__ J1,
    float* __restrict__ J2, unsigned flags, double dt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cell_tile<O, DIM>(G, B, P, J0, J1, J2, flags, dt, xcd_tile(blockIdx.x, gridDim.x), smem_raw);
}

// Charge density on the same tiles: the three component waves take every third particle of
// each cell into three copies of the window (summed by the density window sum).
template <int O, int DIM>
__global__ __launch_bounds__(CV_WAVES * PIC_WAVE, 3) void k_dep_cell_rho(KGrid G, KBins B,
                                                                         KPart P,
                                                                         float* __restrict__ rho) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cell_tile<O, DIM, true>(G, B, P, rho, rho, rho, 0u, 0.0, xcd_tile(blockIdx.x, gridDim.x),
                          smem_raw);
}

// Persistent batched deposition (3D patches, any order): each workgroup pulls (patch,
// tile) items from a device counter until the list is exhausted, so patches of uneven
// size and order share one launch and the longest items (listed first) start first.
__global__ __launch_bounds__(CV_WAVES * PIC_WAVE, 3) void k_dep_cell_batched(
    const BatchPatch* __restrict__ pd, const int2* __restrict__ items, int nitems,
    int* __restrict__ queue, unsigned flags) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= nitems) break;
    const int pi = __builtin_amdgcn_readfirstlane(items[it].x);
    const int tile = __builtin_amdgcn_readfirstlane(items[it].y);
    const BatchPatch& d = pd[pi];
    const int order = d.G.order;
    if (order == 1) cell_tile<1, 3>(d.G, d.B, d.P, d.J[0], d.J[1], d.J[2], flags, d.dt, tile, smem_raw);
    else if (order == 2) cell_tile<2, 3>(d.G, d.B, d.P, d.J[0], d.J[1], d.J[2], flags, d.dt, tile, smem_raw);
    else cell_tile<3, 3>(d.G, d.B, d.P, d.J[0], d.J[1], d.J[2], flags, d.dt, tile, smem_raw);
    __syncthreads();
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

size_t cell_smem_bytes(int order, int dim, const KBins& kb) {
  if (dim == 3) {
    if (order == 1) return CellLayout<1, 3>(kb).total;
    if (order == 2) return CellLayout<2, 3>(kb).total;
    return CellLayout<3, 3>(kb).total;
  }
  if (order == 1) return CellLayout<1, 2>(kb).total;
  if (order == 2) return CellLayout<2, 2>(kb).total;
  return CellLayout<3, 2>(kb).total;
}

int batched_blocks_per_cu(size_t smem) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_dep_cell_batched, CV_WAVES * PIC_WAVE,
                                                   smem) != hipSuccess)
    nb = 1;
  return nb < 1 ? 1 : nb;
}

void batched_cell_launch(const BatchPatch* pd, const int2* items, int nitems, int* queue,
                         int blocks, size_t smem, unsigned flags, hipStream_t s) {
  hipLaunchKernelGGL(k_dep_cell_batched, dim3(blocks), dim3(CV_WAVES * PIC_WAVE), smem, s, pd,
                     items, nitems, queue, flags);
}

template <int O, int DIM>
static bool launch_cell_rho(const KGrid& G, const KPart& P, pic_bins* b, float* rho,
                            hipStream_t s) {
  const size_t smem = CellLayout<O, DIM>(b->kb).total;
  if (smem > b->max_lds) return false;
  hipLaunchKernelGGL((k_dep_cell_rho<O, DIM>), dim3(b->kb.ntiles), dim3(CV_WAVES * PIC_WAVE), smem,
                     s, G, b->kb, P, rho);
  return true;
}

bool deposit_rho_cell_launch(const KGrid& G, const KPart& P, pic_bins* b, float* rho,
                             hipStream_t s) {
#define CR(O_, D_) return launch_cell_rho<O_, D_>(G, P, b, rho, s)
  if (G.dim == 3) {
    if (G.order == 1) CR(1, 3); else if (G.order == 2) CR(2, 3); else CR(3, 3);
  } else {
    if (G.order == 1) CR(1, 2); else if (G.order == 2) CR(2, 2); else CR(3, 2);
  }
#undef CR
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
