// Current deposition kernels (Eq. 1, Sec. 3.1) for gfx950.
//
//  k_dep_unsorted    one particle per lane, global float atomics (no bins; the ablation
//                    of deposition without sorting).
//  k_dep_tile_atomic one workgroup per particle tile: particles of the tile's bins are
//                    read with coalesced loads, their 3 (O+1)^DIM contributions added
//                    with ds_add_f32 into an LDS window covering the tile plus its stencil
//                    halo, and the window is stored once (tile-level reduction, the
//                    rhocell -> grid step of Eq. 5 at tile granularity); k_halo_tile then
//                    adds the overlapping windows of neighbouring tiles into J. Particles whose
//                    cell no longer matches their bin are deposited exactly (LDS when the
//                    stencil fits the window, global atomics otherwise) and, with
//                    PIC_F_EMIT_MOVERS, listed for the next incremental rebin (the mover
//                    detection fused into stage 1 of Alg. 2, Sec. 4.3). With PIC_F_DRIFT
//                    the kernel then advances the position and lists movers against it.
#include "deposit_common.h"

__device__ uint32_t g_pic_err_nobins;

__global__ void k_fill_f32(float* __restrict__ p, int64_t n, float v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

void launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
}

// Zero the three current components in one launch (float4 stores where aligned) and, when
// given, the bins' mover counters.
__global__ void k_zero_j3(float* __restrict__ a, float* __restrict__ b, float* __restrict__ c,
                          int64_t n, int32_t* __restrict__ ctr) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ctr && i0 == 0) {
    ctr[CTR_NMOV] = 0;
    ctr[CTR_NDROP] = 0;
  }
  float* arr[3] = {a, b, c};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float* p = arr[k];
    const int64_t head = (int64_t)((-(((uintptr_t)p) >> 2)) & 3);   // floats before 16-B alignment
    const int64_t h = head < n ? head : n;
    for (int64_t i = i0; i < h; i += stride) p[i] = 0.0f;
    const int64_t nv = (n - h) / 4;
    float4* q = (float4*)(p + h);
    for (int64_t i = i0; i < nv; i += stride) q[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int64_t i = h + 4 * nv + i0; i < n; i += stride) p[i] = 0.0f;
  }
}

void launch_zero_j3(float* a, float* b, float* c, int64_t n, hipStream_t s, int32_t* ctr) {
  if (n <= 0 && !ctr) return;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n / 4 + 255) / 256, 4096));
  hipLaunchKernelGGL(k_zero_j3, dim3((unsigned)blocks), dim3(256), 0, s, a, b, c, n, ctr);
}

uint32_t* nobins_err_ptr() {
  static uint32_t* ptr = nullptr;
  if (!ptr) {
    if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(g_pic_err_nobins)) != hipSuccess) ptr = nullptr;
  }
  return ptr;
}

// -----------------------------------------------------------------------------------
template <int O, int DIM>
__global__ __launch_bounds__(256) void k_dep_unsorted(KGrid G, KPart P, float* __restrict__ J0,
                                                      float* __restrict__ J1,
                                                      float* __restrict__ J2, uint32_t* err,
                                                      int drift, double dt, float hdt) {
  const int stride = gridDim.x * blockDim.x;
  uint32_t bad = 0;
  float* J[3] = {J0, J1, J2};
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < P.nslots; s += stride) {
    if (P.id[s] == PIC_INVALID_ID) continue;
    double pos[3] = {P.x[s], P.y[s], DIM == 3 ? P.z[s] : 0.0};
    const float ux = P.ux[s], uy = P.uy[s], uz = P.uz[s];
    double dp[3] = {pos[0], pos[1], pos[2]};
    if (hdt != 0.0f) midpoint_shift<DIM>(G, dp, ux, uy, uz, hdt);   // time-centred position
    PartPrep<O, DIM> p;
    if (!prep_cell<DIM>(G, dp[0], dp[1], dp[2], p.cell, p.f, bad)) continue;
    prep_amp(G.q, ux, uy, uz, P.w[s], p.amp);
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
    if (drift) {
      drift_one<DIM>(G, pos, ux, uy, uz, dt);
      P.x[s] = pos[0];
      P.y[s] = pos[1];
      if (DIM == 3) P.z[s] = pos[2];
    }
  }
  if (bad) atomicOr(err, bad);
}

// -----------------------------------------------------------------------------------
template <int O, int DIM>
__global__ __launch_bounds__(256) void k_dep_tile_atomic(KGrid G, KBins B, KPart P,
                                                         float* __restrict__ J0,
                                                         float* __restrict__ J1,
                                                         float* __restrict__ J2, unsigned flags,
                                                         double dt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int t = blockIdx.x;
  const TileBox tb = tile_box(G.n, B.T, B.nt, t);
  const TileWin<O, DIM> tw(tb);
  int32_t* s_off = (int32_t*)smem_raw;
  int32_t* s_len = s_off + tb.nb + 1;
  float* win = (float*)(smem_raw + tile_smem_head(B));
  float* J[3] = {J0, J1, J2};

  for (int i = threadIdx.x; i <= tb.nb; i += blockDim.x) s_off[i] = B.off[tb.b0 + i];
  for (int i = threadIdx.x; i < tb.nb; i += blockDim.x) s_len[i] = B.len[tb.b0 + i];
  for (int i = threadIdx.x; i < 3 * tw.size; i += blockDim.x) win[i] = 0.0f;
  __syncthreads();

  const int S0 = s_off[0], S1 = s_off[tb.nb];
  const bool emit = flags & PIC_F_EMIT_MOVERS;
  const bool drift = flags & PIC_F_DRIFT;
  uint32_t bad = 0;
  // Strided slot order: in round r thread t takes slot S0 + r + t * rounds, so the lanes
  // of a wave hold particles of different cells and rarely add to the same LDS word at
  // once (consecutive slots are mostly the same cell).
  const int rounds = (S1 - S0 + (int)blockDim.x - 1) / (int)blockDim.x;
  for (int r = 0; r < rounds; ++r) {
    const int s = S0 + r + (int)threadIdx.x * rounds;
    int lb = 0;
    bool act = s < S1;
    if (act) {
      lb = slot_bin(s_off, tb.nb, s);
      act = s < s_off[lb] + s_len[lb];
    }
    PartPrep<O, DIM> p;
    double pos[3] = {0.0, 0.0, 0.0};
    float ux = 0.f, uy = 0.f, uz = 0.f;
    if (act) {
      pos[0] = P.x[s];
      pos[1] = P.y[s];
      if (DIM == 3) pos[2] = P.z[s];
      act = prep_cell<DIM>(G, pos[0], pos[1], pos[2], p.cell, p.f, bad);
    }
    if (act) {
      ux = P.ux[s];
      uy = P.uy[s];
      uz = P.uz[s];
      prep_amp(G.q, ux, uy, uz, P.w[s], p.amp);
      prep_shapes(p);
      if (tw.fits(p)) {
        scatter_particle(p, [&](int c, int mx, int my, int mz, float v) {
          atomicAdd(&win[tw.index(c, mx, my, mz)], v);
        });
      } else {
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
    int32_t newbin = -1;
    if (act && drift) {
      drift_one<DIM>(G, pos, ux, uy, uz, dt);
      P.x[s] = pos[0];
      P.y[s] = pos[1];
      if (DIM == 3) P.z[s] = pos[2];
    }
    if (emit) {
      bool mv = false;
      if (act) {
        int c2[3];
        float f2[3];
        if (prep_cell<DIM>(G, pos[0], pos[1], pos[2], c2, f2, bad)) {
          newbin = bin_of_cell(G.n, B.T, c2[0], c2[1], c2[2]);
          mv = newbin != tb.b0 + lb;
        }
      }
      int e = wave_append(mv, &B.ctr[CTR_NMOV]);
      if (mv) {
        if (e < B.max_movers) {
          B.mv_slot[e] = s;
          B.mv_old[e] = tb.b0 + lb;
          B.mv_new[e] = newbin;
        } else {
          atomicAdd(&B.ctr[CTR_NDROP], 1);
        }
      }
    }
  }
  if (bad) atomicOr(B.err, bad);
  __syncthreads();
  store_window<O, DIM>(B, t, tw, win, blockDim.x, threadIdx.x);
}

// J += sum of the stored tile windows covering each node (at most 2 tiles per
// dimension for tiles at least as wide as the stencil reach). One thread per node, all
// three components.
// Batched launches: blockIdx.y = patch.
__global__ __launch_bounds__(256) void k_batched_prologue(const BatchPatch* __restrict__ pd,
                                                          int* __restrict__ queue, unsigned flags) {
  const BatchPatch& d = pd[blockIdx.y];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (flags & PIC_F_EMIT_MOVERS) {
      d.B.ctr[CTR_NMOV] = 0;
      d.B.ctr[CTR_NDROP] = 0;
    }
    if (blockIdx.y == 0) *queue = 0;
  }
  if (flags & PIC_F_ACCUMULATE) return;
  const int64_t tot = (int64_t)d.G.N[0] * d.G.N[1] * d.G.N[2];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += stride) {
    d.J[0][i] = 0.0f;
    d.J[1][i] = 0.0f;
    d.J[2][i] = 0.0f;
  }
}

void batched_prologue_launch(const BatchPatch* pd, int npatch, int64_t max_nodes, int* queue,
                             unsigned flags, hipStream_t s) {
  const unsigned bx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((max_nodes + 255) / 256, 512));
  hipLaunchKernelGGL(k_batched_prologue, dim3(bx, npatch), dim3(256), 0, s, pd, queue, flags);
}

// Tile-centric window sum: workgroup t owns the J nodes of its cells (on a guard dimension
// the first and last tiles also own the stencil nodes beyond the domain) and adds, for each
// of them, the entries of every tile window that covers it: its own and, near its faces,
// the neighbours' (periodic neighbours across the boundary shifted by n). The stencil
// reaches at most 2 nodes out; a ragged last tile may be a single cell wide, so tiles up to
// three positions away are examined. Each stored node is written by exactly one workgroup.
// RHO: the three window copies of the charge density are summed into J0.
constexpr int HALO_MAXC = 6;      // candidate windows per dimension
constexpr int HALO_GX = 4;        // tiles along x per workgroup of the single-grid window sum

// The workgroup owns the nodes of gx consecutive tiles along x starting at `tile` (a row
// of tiles: J is then read and written in whole lines); a node's candidate windows and
// their order do not depend on gx.
template <int O, int DIM, bool RHO>
__device__ __forceinline__ void halo_tile_body(const KGrid& G, const KBins& B,
                                               float* __restrict__ J0, float* __restrict__ J1,
                                               float* __restrict__ J2, int tile, int gx,
                                               int32_t* sh) {
  constexpr int LO = TileWin<O, DIM>::LO, R = TileWin<O, DIM>::R;
  const TileBox tb = tile_box(G.n, B.T, B.nt, tile);
  const TileBox tl = tile_box(G.n, B.T, B.nt, tile + gx - 1);   // last tile of the row
  int tcoord[3];
  {
    int t = tile;
    tcoord[0] = t % B.nt[0];
    t /= B.nt[0];
    tcoord[1] = t % B.nt[1];
    tcoord[2] = t / B.nt[1];
  }
  // own node range per dimension
  int a[3], len[3], off[3];
  int tot = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d >= DIM) {
      a[d] = 0;
      len[d] = 1;
    } else {
      const int last = d == 0 ? tcoord[0] + gx - 1 : tcoord[d];
      a[d] = tb.c0[d];
      int b = tl.c0[d] + tl.e[d];
      if (!G.per[d]) {
        if (tcoord[d] == 0) a[d] = tb.c0[d] + LO;
        if (last == B.nt[d] - 1) b = tl.c0[d] + tl.e[d] + R + LO;
      }
      len[d] = b - a[d];
    }
    off[d] = tot;
    tot += len[d];
  }
  // candidates per own coordinate: count, neighbour tile coordinate, window coordinate,
  // window width
  int32_t* s_cnt = sh;
  int32_t* s_t = s_cnt + tot;
  int32_t* s_w = s_t + HALO_MAXC * tot;
  int32_t* s_W = s_w + HALO_MAXC * tot;
  for (int i = threadIdx.x; i < tot; i += blockDim.x) {
    const int d = i >= off[2] ? 2 : (i >= off[1] ? 1 : 0);
    const int m = a[d] + (i - off[d]);
    int cnt = 0;
    if (d >= DIM) {
      s_t[i * HALO_MAXC] = 0;
      s_w[i * HALO_MAXC] = 0;
      s_W[i * HALO_MAXC] = 1;
      cnt = 1;
    } else {
      for (int k = -3; k <= 3 + (d == 0 ? gx - 1 : 0); ++k) {
        int tn = tcoord[d] + k;
        int shift = 0;
        if (tn < 0 || tn >= B.nt[d]) {
          if (!G.per[d]) continue;
          // periodic image: wrap the tile index, shift its cells by whole domains
          const int wraps = tn < 0 ? -((-tn + B.nt[d] - 1) / B.nt[d]) : tn / B.nt[d];
          shift = wraps * G.n[d];
          tn -= wraps * B.nt[d];
        }
        const int c0 = tn * B.T[d] + shift;
        const int e = min(B.T[d], G.n[d] - tn * B.T[d]);
        const int w = m - (c0 + LO);
        if (w >= 0 && w < e + R && cnt < HALO_MAXC) {
          s_t[i * HALO_MAXC + cnt] = tn;
          s_w[i * HALO_MAXC + cnt] = w;
          s_W[i * HALO_MAXC + cnt] = e + R;
          ++cnt;
        }
      }
    }
    s_cnt[i] = cnt;
  }
  __syncthreads();
  const int nn = len[0] * len[1] * len[2];
  for (int q = threadIdx.x; q < nn; q += blockDim.x) {
    const int ix = q % len[0], iy = (q / len[0]) % len[1], iz = q / (len[0] * len[1]);
    const int i0 = off[0] + ix, i1 = off[1] + iy, i2 = off[2] + iz;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
    for (int cz = 0; cz < s_cnt[i2]; ++cz)
      for (int cy = 0; cy < s_cnt[i1]; ++cy)
        for (int cx = 0; cx < s_cnt[i0]; ++cx) {
          const int t = s_t[i0 * HALO_MAXC + cx] +
                        B.nt[0] * (s_t[i1 * HALO_MAXC + cy] + B.nt[1] * s_t[i2 * HALO_MAXC + cz]);
          const int li = (s_w[i2 * HALO_MAXC + cz] * s_W[i1 * HALO_MAXC + cy] +
                          s_w[i1 * HALO_MAXC + cy]) * s_W[i0 * HALO_MAXC + cx] +
                         s_w[i0 * HALO_MAXC + cx];
          const float* src = B.wscr + (int64_t)t * 3 * B.wmax + li;
          s0 += src[0];
          s1 += src[B.wmax];
          s2 += src[2 * B.wmax];
        }
    const int sx = store_idx(G, 0, a[0] + ix), sy = store_idx(G, 1, a[1] + iy);
    const int sz = DIM == 3 ? store_idx(G, 2, a[2] + iz) : 0;
    const int64_t idx = ((int64_t)sz * G.N[1] + sy) * G.N[0] + sx;
    if constexpr (RHO) {
      J0[idx] += (s0 + s1) + s2;
    } else {
      J0[idx] += s0;
      J1[idx] += s1;
      J2[idx] += s2;
    }
  }
}

template <int O, int DIM, bool RHO>
__global__ __launch_bounds__(256) void k_halo_tile(KGrid G, KBins B, float* __restrict__ J0,
                                                   float* __restrict__ J1,
                                                   float* __restrict__ J2) {
  extern __shared__ __align__(16) int32_t sh[];
  // workgroup -> row of up to HALO_GX tiles along x (rows in the tiles' XCD order)
  const int ngx = (B.nt[0] + HALO_GX - 1) / HALO_GX;
  const int g = xcd_tile(blockIdx.x, gridDim.x);
  const int gxi = g % ngx, rest = g / ngx;
  const int t0 = gxi * HALO_GX + B.nt[0] * rest;
  halo_tile_body<O, DIM, RHO>(G, B, J0, J1, J2, t0, min(HALO_GX, B.nt[0] - gxi * HALO_GX), sh);
}

// Batched window sum: one workgroup per (patch, first tile of a row of up to HALO_GX tiles
// along x) item of the plan.
__global__ __launch_bounds__(256) void k_batched_halo_tile(const BatchPatch* __restrict__ pd,
                                                           const int2* __restrict__ items) {
  extern __shared__ __align__(16) int32_t sh[];
  const int pi = __builtin_amdgcn_readfirstlane(items[blockIdx.x].x);
  const int tile = __builtin_amdgcn_readfirstlane(items[blockIdx.x].y);
  const BatchPatch& d = pd[pi];
  const int gx = min(HALO_GX, d.B.nt[0] - tile % d.B.nt[0]);
  if (d.G.order == 1) halo_tile_body<1, 3, false>(d.G, d.B, d.J[0], d.J[1], d.J[2], tile, gx, sh);
  else if (d.G.order == 2) halo_tile_body<2, 3, false>(d.G, d.B, d.J[0], d.J[1], d.J[2], tile, gx, sh);
  else halo_tile_body<3, 3, false>(d.G, d.B, d.J[0], d.J[1], d.J[2], tile, gx, sh);
}

size_t halo_smem_bytes(const KBins& kb) {
  int tot = 0;
  for (int d = 0; d < 3; ++d) tot += (d == 0 ? HALO_GX : 1) * kb.T[d] + 4;
  return (size_t)tot * (1 + 3 * HALO_MAXC) * sizeof(int32_t);
}

int halo_row_tiles() { return HALO_GX; }

void batched_halo_tile_launch(const BatchPatch* pd, const int2* items, int nitems, size_t smem,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_batched_halo_tile, dim3(nitems), dim3(256), smem, s, pd, items);
}

template <int O, int DIM, bool RHO>
static void launch_halo_tile(const KGrid& G, pic_bins* b, float* J0, float* J1, float* J2,
                             hipStream_t s) {
  int tot = 0;
  for (int d = 0; d < 3; ++d)
    tot += d < DIM ? (d == 0 ? HALO_GX : 1) * b->kb.T[d] + TileWin<O, DIM>::R : 1;
  const size_t smem = (size_t)tot * (1 + 3 * HALO_MAXC) * sizeof(int32_t);
  const int ngx = (b->kb.nt[0] + HALO_GX - 1) / HALO_GX;
  const int groups = ngx * b->kb.nt[1] * b->kb.nt[2];
  hipLaunchKernelGGL((k_halo_tile<O, DIM, RHO>), dim3(groups), dim3(256), smem, s, G, b->kb,
                     J0, J1, J2);
}

void halo_rho_launch(const KGrid& G, pic_bins* b, float* rho, hipStream_t s) {
#define HR(O_, D_) launch_halo_tile<O_, D_, true>(G, b, rho, rho, rho, s)
  if (G.dim == 3) {
    if (G.order == 1) HR(1, 3); else if (G.order == 2) HR(2, 3); else HR(3, 3);
  } else {
    if (G.order == 1) HR(1, 2); else if (G.order == 2) HR(2, 2); else HR(3, 2);
  }
#undef HR
}

void halo_launch(const KGrid& G, pic_bins* b, float* J0, float* J1, float* J2, hipStream_t s) {
#define HL(O_, D_) launch_halo_tile<O_, D_, false>(G, b, J0, J1, J2, s)
  if (G.dim == 3) {
    if (G.order == 1) HL(1, 3); else if (G.order == 2) HL(2, 3); else HL(3, 3);
  } else {
    if (G.order == 1) HL(1, 2); else if (G.order == 2) HL(2, 2); else HL(3, 2);
  }
#undef HL
}

// -----------------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(256) void k_drift(KGrid G, KPart P, double dt) {
  const int stride = gridDim.x * blockDim.x;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < P.nslots; s += stride) {
    if (P.id[s] == PIC_INVALID_ID) continue;
    double pos[3] = {P.x[s], P.y[s], DIM == 3 ? P.z[s] : 0.0};
    drift_one<DIM>(G, pos, P.ux[s], P.uy[s], P.uz[s], dt);
    P.x[s] = pos[0];
    P.y[s] = pos[1];
    if (DIM == 3) P.z[s] = pos[2];
  }
}

void drift_launch(const KGrid& G, const KPart& P, double dt, hipStream_t s) {
  if (P.nslots <= 0) return;
  unsigned blocks = (unsigned)std::min<int64_t>(((int64_t)P.nslots + 255) / 256, 16384);
  if (G.dim == 3) hipLaunchKernelGGL(k_drift<3>, dim3(blocks), dim3(256), 0, s, G, P, dt);
  else hipLaunchKernelGGL(k_drift<2>, dim3(blocks), dim3(256), 0, s, G, P, dt);
}

// -----------------------------------------------------------------------------------
template <int O, int DIM>
static void launch_unsorted(const KGrid& G, const KPart& P, float* J0, float* J1, float* J2,
                            uint32_t* err, bool drift, double dt, float hdt, hipStream_t s) {
  unsigned blocks = (unsigned)std::min<int64_t>(((int64_t)P.nslots + 255) / 256, 16384);
  if (blocks == 0) return;
  hipLaunchKernelGGL((k_dep_unsorted<O, DIM>), dim3(blocks), dim3(256), 0, s, G, P, J0, J1, J2,
                     err, drift ? 1 : 0, dt, hdt);
}

template <int O, int DIM>
static bool launch_tile_atomic(const KGrid& G, const KPart& P, pic_bins* b, float* J0,
                               float* J1, float* J2, unsigned flags, double dt, hipStream_t s) {
  size_t smem = tile_smem_head(b->kb) + 3 * sizeof(float) * TileWin<O, DIM>::max_size(b->kb);
  if (smem > b->max_lds) return false;
  hipLaunchKernelGGL((k_dep_tile_atomic<O, DIM>), dim3(b->kb.ntiles), dim3(256), smem, s, G,
                     b->kb, P, J0, J1, J2, flags, dt);
  return true;
}

bool deposit_launch(const KGrid& G, const KPart& P, pic_bins* b, float* J0, float* J1, float* J2,
                    int path, unsigned flags, double dt, hipStream_t s) {
  int64_t nJ = (int64_t)G.N[0] * G.N[1] * G.N[2];
  const bool emit = b && (flags & PIC_F_EMIT_MOVERS);
  if (!(flags & PIC_F_ACCUMULATE)) launch_zero_j3(J0, J1, J2, nJ, s, emit ? b->kb.ctr : nullptr);
  else if (emit) reset_movers(b, s);
  const bool drift = flags & PIC_F_DRIFT;
  if (!b) {
    uint32_t* err = nobins_err_ptr();
    const float hdt = !(flags & PIC_F_MIDPOINT) ? 0.0f : (float)(drift ? 0.5 * dt : -0.5 * dt);
#define UNS(O_, D_) launch_unsorted<O_, D_>(G, P, J0, J1, J2, err, drift, dt, hdt, s)
    if (G.dim == 3) {
      if (G.order == 1) UNS(1, 3); else if (G.order == 2) UNS(2, 3); else UNS(3, 3);
    } else {
      if (G.order == 1) UNS(1, 2); else if (G.order == 2) UNS(2, 2); else UNS(3, 2);
    }
#undef UNS
    return true;
  }
  if (path == PIC_PATH_AUTO) path = choose_path(G, b);
  bool ok = false;
  if (path == PIC_PATH_CELL_VALU || path == PIC_PATH_MFMA_BF16 || path == PIC_PATH_MFMA_FP16) {
    ok = deposit_cell_launch(G, P, b, J0, J1, J2, path, flags, dt, s);
  } else {
#define TIL(O_, D_) ok = launch_tile_atomic<O_, D_>(G, P, b, J0, J1, J2, flags, dt, s)
    if (G.dim == 3) {
      if (G.order == 1) TIL(1, 3); else if (G.order == 2) TIL(2, 3); else TIL(3, 3);
    } else {
      if (G.order == 1) TIL(1, 2); else if (G.order == 2) TIL(2, 2); else TIL(3, 2);
    }
#undef TIL
  }
  if (ok) halo_launch(G, b, J0, J1, J2, s);
  return ok;
}
