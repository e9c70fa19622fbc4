// Split-precision MFMA deposition: the outer-product formulation of Sec. 4.2.1 (Eq. 7 and
// the two-particle / third-order extensions) mapped onto gfx950 matrix cores.
//
// For a run of consecutive cells along x (a row segment of at most 16 - R cells, R the
// stencil reach) every particle's contribution to component c is the rank-1 tensor
//     (amp_c s_x) (x) (s_y (x) s_z),
// so the segment's current is one matrix product over K = its particles:
//     J_c[x-node, (y,z)-node] = sum_p A_c[x-node, p] B_c[p, (y,z)-node],
// A_c holding amp_c s_x of each particle placed at its x offset inside the segment's
// 16-node x window (the particles of all cells of the segment share one output tile), and
// B_c the s_y s_z products on the y/z stencil window (16 or 20 nodes, one or two 16-wide
// N tiles). One v_mfma_f32_16x16x32 per split product and N tile handles 32 particles.
//
// Precision: each float32 operand v is split into hi = round(v) and lo = round(v - hi)
// (bf16, or fp16 with lo scaled by 2^11 so it stays normal); hi*hi + hi*lo + lo*hi are
// accumulated in float32 by the matrix core, leaving about 2^-16 relative error per
// product (bf16) or 2^-22 (fp16).
//
// One wave per tile: lanes = slots build the operands (position -> cell in FP64, the
// fused drift and mover detection as in the per-cell path), a wave-local LDS staging
// area feeds the MFMAs, and each segment's output tiles are added to the tile's LDS
// window with plain read-add-write (every lane holds distinct nodes; segments are
// processed in order by the same wave).
#include "deposit_common.h"

typedef __bf16 v8bf16 __attribute__((ext_vector_type(8)));
typedef _Float16 v8f16 __attribute__((ext_vector_type(8)));
typedef float v4f32 __attribute__((ext_vector_type(4)));
typedef float v2f32 __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf16 __attribute__((ext_vector_type(2)));
typedef _Float16 v2f16 __attribute__((ext_vector_type(2)));

template <int O, int DIM>
__host__ __device__ constexpr int mw(int c, int d) {
  return d < DIM ? win_w(O, c == d) : 1;
}
template <int O, int DIM>
__host__ __device__ constexpr int mN(int c) {
  return mw<O, DIM>(c, 1) * mw<O, DIM>(c, 2);
}
template <int O, int DIM>
__host__ __device__ constexpr int mNT(int c) {
  return (mN<O, DIM>(c) + 15) / 16;
}
// First B column of component c.
template <int O, int DIM>
__host__ __device__ constexpr int mCol(int c) {
  return 16 * ((c > 0 ? mNT<O, DIM>(0) : 0) + (c > 1 ? mNT<O, DIM>(1) : 0));
}
template <int O, int DIM>
__host__ __device__ constexpr int mCols() {
  return mCol<O, DIM>(3 - 1) + 16 * mNT<O, DIM>(2);
}

constexpr int MK = 64;  // particle slots staged per batch (two K = 32 chunks)

template <int O, int DIM>
struct MfmaStage {
  uint16_t ah[3][16][MK];
  uint16_t al[3][16][MK];
  uint16_t bh[mCols<O, DIM>()][MK];
  uint16_t bl[mCols<O, DIM>()][MK];
};

// hi/lo split of a float32 value into two 16-bit patterns.
template <bool BF>
__device__ __forceinline__ void split16(float v, uint16_t& hi, uint16_t& lo) {
  if constexpr (BF) {
    v2f32 x = {v, 0.0f};
    v2bf16 h = __builtin_convertvector(x, v2bf16);
    v2f32 hf = __builtin_convertvector(h, v2f32);
    v2f32 r = {v - hf[0], 0.0f};
    v2bf16 l = __builtin_convertvector(r, v2bf16);
    hi = __builtin_bit_cast(uint16_t, h[0]);
    lo = __builtin_bit_cast(uint16_t, l[0]);
  } else {
    _Float16 h = (_Float16)v;
    _Float16 l = (_Float16)((v - (float)h) * 2048.0f);
    hi = __builtin_bit_cast(uint16_t, h);
    lo = __builtin_bit_cast(uint16_t, l);
  }
}

template <bool BF>
__device__ __forceinline__ v4f32 mfma(const uint16_t* a, const uint16_t* b, v4f32 c) {
  if constexpr (BF) {
    v8bf16 av = *(const v8bf16*)a;
    v8bf16 bv = *(const v8bf16*)b;
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
  } else {
    v8f16 av = *(const v8f16*)a;
    v8f16 bv = *(const v8f16*)b;
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, c, 0, 0, 0);
  }
}

// Byte offset of the staging area: after the bin tables and the window, 16-byte aligned
// (the MFMA operands are read with 128-bit LDS loads).
template <int O, int DIM>
__host__ __device__ __forceinline__ size_t mfma_stage_off(const KBins& kb) {
  return (tile_smem_head(kb) + 3 * sizeof(float) * TileWin<O, DIM>::max_size(kb) + 15) &
         ~(size_t)15;
}

template <int O, int DIM, bool BF>
__global__ __launch_bounds__(PIC_WAVE) void k_dep_mfma(KGrid G, KBins B, KPart P,
                                                       float* __restrict__ J0,
                                                       float* __restrict__ J1,
                                                       float* __restrict__ J2, unsigned flags,
                                                       double dt) {
  constexpr int LO = TileWin<O, DIM>::LO, R = TileWin<O, DIM>::R;
  constexpr int SW = 16 - R;                       // cells per row segment
  constexpr int NT0 = mNT<O, DIM>(0), NT1 = mNT<O, DIM>(1), NT2 = mNT<O, DIM>(2);
  constexpr int NTT = NT0 + NT1 + NT2;             // output tiles per segment
  constexpr int WN = win_w(O, false), WS = win_w(O, true);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int t = blockIdx.x;
  const TileBox tb = tile_box(G.n, B.T, B.nt, t);
  const TileWin<O, DIM> tw(tb);
  int32_t* s_off = (int32_t*)smem_raw;
  int32_t* s_len = s_off + tb.nb + 1;
  float* win = (float*)(smem_raw + tile_smem_head(B));
  MfmaStage<O, DIM>& st = *(MfmaStage<O, DIM>*)(smem_raw + mfma_stage_off<O, DIM>(B));
  float* J[3] = {J0, J1, J2};
  const int lane = threadIdx.x;
  for (int i = lane; i <= tb.nb; i += PIC_WAVE) s_off[i] = B.off[tb.b0 + i];
  for (int i = lane; i < tb.nb; i += PIC_WAVE) s_len[i] = B.len[tb.b0 + i];
  for (int i = lane; i < 3 * tw.size; i += PIC_WAVE) win[i] = 0.0f;
  {
    uint32_t* z = (uint32_t*)&st;
    for (int i = lane; i < (int)(sizeof(MfmaStage<O, DIM>) / 4); i += PIC_WAVE) z[i] = 0u;
  }
  __syncthreads();
  const bool emit = flags & PIC_F_EMIT_MOVERS;
  const bool drift = flags & PIC_F_DRIFT;
  uint32_t bad = 0;
  const int ex = tb.e[0], ey = tb.e[1], ez = tb.e[2];
  const int m16 = lane & 15, g4 = lane >> 4;

  for (int rz = 0; rz < ez; ++rz)
    for (int ry = 0; ry < ey; ++ry)
      for (int sx = 0; sx < ex; sx += SW) {
        const int sn = min(SW, ex - sx);             // cells in the segment
        const int cb = (rz * ey + ry) * ex + sx;     // first local bin
        const int S0 = s_off[cb], S1 = s_off[cb + sn];
        const int gx0 = tb.c0[0] + sx;               // first cell x of the segment
        const int cy = tb.c0[1] + ry, cz = tb.c0[2] + rz;
        v4f32 acc[NTT], acc2[NTT];
#pragma unroll
        for (int q = 0; q < NTT; ++q) {
          acc[q] = (v4f32){0.f, 0.f, 0.f, 0.f};
          acc2[q] = (v4f32){0.f, 0.f, 0.f, 0.f};
        }
        for (int base = S0; base < S1; base += MK) {
          const int s = base + lane;
          int lb = cb;
          bool act = s < S1;
          if (act) {
            while (lb + 1 < cb + sn && s_off[lb + 1] <= s) ++lb;
            act = s < s_off[lb] + s_len[lb];
          }
          PartPrep<O, DIM> p;
          double pos[3] = {0.0, 0.0, 0.0};
          float ux = 0.f, uy = 0.f, uz = 0.f;
          bool ok = false, mine = false;
          if (act) {
            pos[0] = P.x[s];
            pos[1] = P.y[s];
            if (DIM == 3) pos[2] = P.z[s];
            ok = prep_cell<DIM>(G, pos[0], pos[1], pos[2], p.cell, p.f, bad);
          }
          if (ok) {
            ux = P.ux[s];
            uy = P.uy[s];
            uz = P.uz[s];
            prep_amp(G.q, ux, uy, uz, P.w[s], p.amp);
            prep_shapes(p);
            mine = p.cell[0] == gx0 + (lb - cb) && p.cell[1] == cy && (DIM == 2 || p.cell[2] == cz);
            if (!mine) {
              // stale particle: exact per-particle path through global atomics
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
          // operands of this lane's slot (column `lane` of the staging area)
          if (mine) {
            float wnp[3][WN], wsp[3][WS];
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
#pragma unroll
              for (int a = 0; a < WN; ++a) {
                float v0 = a <= O ? p.wn[d][a <= O ? a : 0] : 0.f;
                float v1 = (a >= 1 && a - 1 <= O) ? p.wn[d][(a >= 1 && a - 1 <= O) ? a - 1 : 0] : 0.f;
                wnp[d][a] = p.sn[d] ? v1 : v0;
              }
#pragma unroll
              for (int a = 0; a < WS; ++a) {
                float v0 = a <= O ? p.ws[d][a <= O ? a : 0] : 0.f;
                float v1 = (a >= 1 && a - 1 <= O) ? p.ws[d][(a >= 1 && a - 1 <= O) ? a - 1 : 0] : 0.f;
                wsp[d][a] = p.ss[d] ? v1 : v0;
              }
            }
            if constexpr (DIM == 2) {
              wnp[2][0] = 1.0f;
              wsp[2][0] = 1.0f;
            }
            const int xoff = p.cell[0] - gx0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const int WX = mw<O, DIM>(c, 0), WY = mw<O, DIM>(c, 1), WZ = mw<O, DIM>(c, 2);
              const float* wx = (c == 0) ? wsp[0] : wnp[0];
              const float* wy = (c == 1 && DIM >= 2) ? wsp[1] : wnp[1];
              const float* wz = (c == 2 && DIM == 3) ? wsp[2] : wnp[2];
              const int r0 = xoff + win_lo(O, c == 0) - LO;
#pragma unroll
              for (int a = 0; a < WX; ++a) {
                uint16_t h, l;
                split16<BF>(p.amp[c] * wx[a], h, l);
                st.ah[c][r0 + a][lane] = h;
                st.al[c][r0 + a][lane] = l;
              }
              const int col0 = mCol<O, DIM>(c);
#pragma unroll
              for (int iz = 0; iz < WZ; ++iz)
#pragma unroll
                for (int iy = 0; iy < WY; ++iy) {
                  uint16_t h, l;
                  split16<BF>(wy[iy] * wz[iz], h, l);
                  st.bh[col0 + iz * WY + iy][lane] = h;
                  st.bl[col0 + iz * WY + iy][lane] = l;
                }
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
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          // contraction over the batch: two K = 32 chunks, three split products each
#pragma unroll
          for (int q = 0; q < MK / 32; ++q) {
            const int k0 = q * 32 + g4 * 8;
            int tix = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const uint16_t* ah = &st.ah[c][m16][k0];
              const uint16_t* al = &st.al[c][m16][k0];
              const int ntc = c == 0 ? NT0 : (c == 1 ? NT1 : NT2);
#pragma unroll
              for (int nt = 0; nt < ntc; ++nt) {
                const int col = mCol<O, DIM>(c) + nt * 16 + m16;
                const uint16_t* bh = &st.bh[col][k0];
                const uint16_t* bl = &st.bl[col][k0];
                acc[tix] = mfma<BF>(ah, bh, acc[tix]);
                if constexpr (BF) {
                  acc[tix] = mfma<BF>(ah, bl, acc[tix]);
                  acc[tix] = mfma<BF>(al, bh, acc[tix]);
                } else {
                  acc2[tix] = mfma<BF>(ah, bl, acc2[tix]);
                  acc2[tix] = mfma<BF>(al, bh, acc2[tix]);
                }
                ++tix;
              }
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          // clear the A planes for the next batch (B columns are overwritten or unused)
          {
            uint4* z = (uint4*)&st.ah[0][0][0];
            const int n16 = (int)(2 * sizeof(st.ah) / 16);
            for (int i = lane; i < n16; i += PIC_WAVE) z[i] = make_uint4(0u, 0u, 0u, 0u);
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // output tile (4 rows x 1 column per lane) -> tile window, read-add-write
        {
          int tix = 0;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const int WY = mw<O, DIM>(c, 1);
            const int ntc = c == 0 ? NT0 : (c == 1 ? NT1 : NT2);
            const int ylo = DIM >= 2 ? cy + win_lo(O, c == 1) : 0;
            const int zlo = DIM == 3 ? cz + win_lo(O, c == 2) : 0;
#pragma unroll
            for (int nt = 0; nt < ntc; ++nt) {
              const int n = nt * 16 + m16;
              if (n < mN<O, DIM>(c)) {
                const int iy = n % WY, iz = n / WY;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const int mrow = g4 * 4 + i;
                  const int xn = gx0 + LO + mrow;
                  if (mrow < sn + R) {
                    float v = acc[tix][i];
                    if constexpr (!BF) v += acc2[tix][i] * (1.0f / 2048.0f);
                    const int wi = tw.index(c, xn, ylo + iy, zlo + iz);
                    win[wi] = win[wi] + v;
                  }
                }
              }
              ++tix;
            }
          }
          asm volatile("" ::: "memory");
        }
      }
  if (bad) atomicOr(B.err, bad);
  __syncthreads();
  store_window<O, DIM>(B, t, tw, win, PIC_WAVE, lane);
}

template <int O, int DIM, bool BF>
static bool launch_mfma(const KGrid& G, const KPart& P, pic_bins* b, float* J0, float* J1,
                        float* J2, unsigned flags, double dt, hipStream_t s) {
  size_t smem = mfma_stage_off<O, DIM>(b->kb) + sizeof(MfmaStage<O, DIM>);
  if (smem > b->max_lds) return false;
  hipLaunchKernelGGL((k_dep_mfma<O, DIM, BF>), dim3(b->kb.ntiles), dim3(PIC_WAVE), smem, s, G,
                     b->kb, P, J0, J1, J2, flags, dt);
  return true;
}

bool deposit_mfma_launch(const KGrid& G, const KPart& P, pic_bins* b, float* J0, float* J1,
                         float* J2, int path, unsigned flags, double dt, hipStream_t s) {
  const bool bf = path == PIC_PATH_MFMA_BF16;
#define MF(O_, D_)                                                                   \
  return bf ? launch_mfma<O_, D_, true>(G, P, b, J0, J1, J2, flags, dt, s)           \
            : launch_mfma<O_, D_, false>(G, P, b, J0, J1, J2, flags, dt, s)
  if (G.dim == 3) {
    if (G.order == 1) MF(1, 3); else if (G.order == 2) MF(2, 3); else MF(3, 3);
  } else {
    if (G.order == 1) MF(1, 2); else if (G.order == 2) MF(2, 2); else MF(3, 2);
  }
#undef MF
}
