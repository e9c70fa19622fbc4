// Adjoint of the deposition: for L = sum_c <G_c, J_c> every particle gathers G with the
// same shape factors (recomputed, not stored) and their derivatives. The gather is the
// field-interpolation pattern of Sec. 3.1 run backwards through Eq. 1:
//   g_c      = sum_nodes G_c * S_c                      (S_c = s_x s_y s_z, staggered on c)
//   h_{c,d}  = sum_nodes G_c * dS_c/dxi_d
//   dL/dw    = q * sum_c v_c g_c
//   dL/du_b  = q W (g_b / gamma - u_b (sum_c u_c g_c) / gamma^3)
//   dL/dx_d  = q W sum_c v_c h_{c,d} * inv_dx_d
#include <algorithm>

#include "deposit_common.h"
#include "tile_particles.h"

uint32_t* nobins_err_ptr();

// One particle: outputs of slot s. `fetch(c, mx, my, mz, w)` returns G_c at unwrapped node
// (mx, my, mz); `w` is the node's weight product, used only to flag a stencil node outside
// the stored grid.
template <int O, int DIM, class Fetch>
__device__ __forceinline__ void bwd_particle(const KGrid& G, const KPart& P, int s,
                                             const int* cell, const float* f, Fetch&& fetch,
                                             float* __restrict__ dx, float* __restrict__ dy,
                                             float* __restrict__ dz, float* __restrict__ dux,
                                             float* __restrict__ duy, float* __restrict__ duz,
                                             float* __restrict__ dw) {
  constexpr int KZ = DIM == 3 ? O + 1 : 1;
  float r_dx[3] = {0.f, 0.f, 0.f}, r_du[3] = {0.f, 0.f, 0.f};
  const float u[3] = {P.ux[s], P.uy[s], P.uz[s]};
  const float wq = P.w[s] * G.q;
  const float ig = 1.0f / sqrtf(1.0f + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
  float gsum[3], h[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float W[3][O + 1], D[3][O + 1];
    int bse[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d < DIM) {
        int sh;
        if (d == c) {
          sh = shape_w<O, true>(f[d], W[d]);
          (void)shape_dw<O, true>(f[d], D[d]);
          bse[d] = cell[d] + win_lo(O, true) + sh;
        } else {
          sh = shape_w<O, false>(f[d], W[d]);
          (void)shape_dw<O, false>(f[d], D[d]);
          bse[d] = cell[d] + win_lo(O, false) + sh;
        }
      } else {
#pragma unroll
        for (int k = 0; k <= O; ++k) {
          W[d][k] = k == 0 ? 1.0f : 0.0f;
          D[d][k] = 0.0f;
        }
        bse[d] = 0;
      }
    }
    float g = 0.f, hx = 0.f, hy = 0.f, hz = 0.f;
#pragma unroll
    for (int kz = 0; kz < KZ; ++kz) {
#pragma unroll
      for (int ky = 0; ky <= O; ++ky) {
        float sx = 0.f, dsx = 0.f;
#pragma unroll
        for (int kx = 0; kx <= O; ++kx) {
          const float gv = fetch(c, bse[0] + kx, bse[1] + ky, bse[2] + kz,
                                 W[0][kx] * W[1][ky] * W[2][kz]);
          sx += gv * W[0][kx];
          dsx += gv * D[0][kx];
        }
        g += W[2][kz] * W[1][ky] * sx;
        hx += W[2][kz] * W[1][ky] * dsx;
        hy += W[2][kz] * D[1][ky] * sx;
        hz += D[2][kz] * W[1][ky] * sx;
      }
    }
    gsum[c] = g;
    h[c][0] = hx;
    h[c][1] = hy;
    h[c][2] = hz;
  }
  const float v[3] = {u[0] * ig, u[1] * ig, u[2] * ig};
  const float r_dw = G.q * (v[0] * gsum[0] + v[1] * gsum[1] + v[2] * gsum[2]);
  const float ug = u[0] * gsum[0] + u[1] * gsum[1] + u[2] * gsum[2];
  const float ig3 = ig * ig * ig;
#pragma unroll
  for (int b = 0; b < 3; ++b) r_du[b] = wq * (gsum[b] * ig - u[b] * ug * ig3);
#pragma unroll
  for (int d = 0; d < DIM; ++d)
    r_dx[d] = wq * (v[0] * h[0][d] + v[1] * h[1][d] + v[2] * h[2][d]) * G.inv_dxf[d];
  dx[s] = r_dx[0];
  dy[s] = r_dx[1];
  if (DIM == 3) dz[s] = r_dx[2];
  dux[s] = r_du[0];
  duy[s] = r_du[1];
  duz[s] = r_du[2];
  if (dw) dw[s] = r_dw;
}

__device__ __forceinline__ void bwd_zero(int s, int dim, float* dx, float* dy, float* dz,
                                         float* dux, float* duy, float* duz, float* dw) {
  dx[s] = 0.f;
  dy[s] = 0.f;
  if (dim == 3) dz[s] = 0.f;
  dux[s] = 0.f;
  duy[s] = 0.f;
  duz[s] = 0.f;
  if (dw) dw[s] = 0.f;
}

// Global gather of G_c at an unwrapped node (periodic wrap or guard offset).
struct GlobalFetch {
  const KGrid& G;
  const float* const* Gs;
  uint32_t& bad;
  __device__ __forceinline__ float operator()(int c, int mx, int my, int mz, float w) const {
    const int ix = store_idx(G, 0, mx), iy = store_idx(G, 1, my);
    const int iz = G.dim == 3 ? store_idx(G, 2, mz) : 0;
    if ((ix | iy | iz) >= 0) return Gs[c][((int64_t)iz * G.N[1] + iy) * G.N[0] + ix];
    if (w != 0.f) bad |= PIC_EF_STENCIL;
    return 0.f;
  }
};

// Particle-parallel gather (no bins, or particles outside their tile).
template <int O, int DIM>
__global__ __launch_bounds__(256) void k_backward(KGrid G, KPart P, const float* __restrict__ G0,
                                                  const float* __restrict__ G1,
                                                  const float* __restrict__ G2,
                                                  float* __restrict__ dx, float* __restrict__ dy,
                                                  float* __restrict__ dz, float* __restrict__ dux,
                                                  float* __restrict__ duy, float* __restrict__ duz,
                                                  float* __restrict__ dw, uint32_t* err) {
  const float* Gs[3] = {G0, G1, G2};
  uint32_t bad = 0;
  const GlobalFetch gf{G, Gs, bad};
  const int stride = gridDim.x * blockDim.x;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < P.nslots; s += stride) {
    int cell[3];
    float f[3];
    const bool ok = P.id[s] != PIC_INVALID_ID &&
                    prep_cell<DIM>(G, P.x[s], P.y[s], DIM == 3 ? P.z[s] : 0.0, cell, f, bad);
    if (ok) bwd_particle<O, DIM>(G, P, s, cell, f, gf, dx, dy, dz, dux, duy, duz, dw);
    else bwd_zero(s, DIM, dx, dy, dz, dux, duy, duz, dw);
  }
  if (bad) atomicOr(err, bad);
}

// Tiled gather: one workgroup per particle tile loads the tile's stencil window of G (all
// three components) into LDS once, then its particles gather from LDS. A particle whose
// cell is not in the tile (its bin is stale) is listed for k_backward_list. Block ntiles
// clears the outputs of the slots past the last bin.
template <int O, int DIM>
__global__ __launch_bounds__(256) void k_backward_tile(KGrid G, KBins B, KPart P,
                                                       const float* __restrict__ G0,
                                                       const float* __restrict__ G1,
                                                       const float* __restrict__ G2,
                                                       float* __restrict__ dx, float* __restrict__ dy,
                                                       float* __restrict__ dz, float* __restrict__ dux,
                                                       float* __restrict__ duy, float* __restrict__ duz,
                                                       float* __restrict__ dw,
                                                       int32_t* __restrict__ list) {
  extern __shared__ __align__(16) float sG[];
  const float* Gs[3] = {G0, G1, G2};
  uint32_t bad = 0;
  if (blockIdx.x >= (unsigned)B.ntiles) {
    const int stride = TAIL_BLOCKS * blockDim.x;
    for (int s = B.off[B.nbins] + (blockIdx.x - B.ntiles) * blockDim.x + threadIdx.x;
         s < P.nslots; s += stride)
      bwd_zero(s, DIM, dx, dy, dz, dux, duy, duz, dw);
    return;
  }
  const TileBox tb = tile_box(G.n, B.T, B.nt, blockIdx.x);
  const TileWin<O, DIM> tw(tb);
  for (int i = threadIdx.x; i < 3 * tw.size; i += blockDim.x) {
    const int c = i / tw.size;
    const int r = i - c * tw.size;
    const int W01 = tw.W[0] * tw.W[1];
    const int wz = r / W01, wy = (r - wz * W01) / tw.W[0], wx = r - wz * W01 - wy * tw.W[0];
    const int ix = store_idx(G, 0, tw.o[0] + wx), iy = store_idx(G, 1, tw.o[1] + wy);
    const int iz = DIM == 3 ? store_idx(G, 2, tw.o[2] + wz) : 0;
    sG[i] = (ix | iy | iz) >= 0 ? Gs[c][((int64_t)iz * G.N[1] + iy) * G.N[0] + ix] : 0.f;
  }
  __syncthreads();
  auto lf = [&](int c, int mx, int my, int mz, float) -> float {
    return sG[tw.index(c, mx, my, mz)];
  };
  int* pre = (int*)(sG + 3 * tw.size);
  const int nval = tile_valid_prefix(B, tb, pre, pre + tb.nb + 1);
  // gap slots get zeros
  const int S0 = B.off[tb.b0], S1 = B.off[tb.b0 + tb.nb];
  for (int s = S0 + threadIdx.x; s < S1; s += blockDim.x)
    if (P.id[s] == PIC_INVALID_ID) bwd_zero(s, DIM, dx, dy, dz, dux, duy, duz, dw);
  // uniform trip count: every lane reaches the wave-level list append
  for (int base = 0; base < nval; base += blockDim.x) {
    const int j = base + threadIdx.x;
    const int s = j < nval ? tile_valid_slot(B, tb, pre, j) : 0;
    int cell[3];
    float f[3];
    const bool ok = j < nval &&
                    prep_cell<DIM>(G, P.x[s], P.y[s], DIM == 3 ? P.z[s] : 0.0, cell, f, bad);
    const bool local = ok && tw.fits_cell(cell);
    if (local) bwd_particle<O, DIM>(G, P, s, cell, f, lf, dx, dy, dz, dux, duy, duz, dw);
    else if (j < nval && !ok) bwd_zero(s, DIM, dx, dy, dz, dux, duy, duz, dw);
    const int e = wave_append(ok && !local, &B.ctr[CTR_TOTAL]);
    if (e >= 0) list[e] = s;
  }
  if (bad) atomicOr(B.err, bad);
}

// The particles the tiled gather listed (cell outside their tile), from global memory.
template <int O, int DIM>
__global__ __launch_bounds__(256) void k_backward_list(KGrid G, KBins B, KPart P,
                                                       const float* __restrict__ G0,
                                                       const float* __restrict__ G1,
                                                       const float* __restrict__ G2,
                                                       float* __restrict__ dx, float* __restrict__ dy,
                                                       float* __restrict__ dz, float* __restrict__ dux,
                                                       float* __restrict__ duy, float* __restrict__ duz,
                                                       float* __restrict__ dw,
                                                       const int32_t* __restrict__ list) {
  const float* Gs[3] = {G0, G1, G2};
  uint32_t bad = 0;
  const GlobalFetch gf{G, Gs, bad};
  const int n = B.ctr[CTR_TOTAL];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int s = list[e];
    int cell[3];
    float f[3];
    if (prep_cell<DIM>(G, P.x[s], P.y[s], DIM == 3 ? P.z[s] : 0.0, cell, f, bad))
      bwd_particle<O, DIM>(G, P, s, cell, f, gf, dx, dy, dz, dux, duy, duz, dw);
  }
  if (bad) atomicOr(B.err, bad);
}

template <int O, int DIM>
static void launch_bwd(const KGrid& G, const KPart& P, uint32_t* err, const float* G0,
                       const float* G1, const float* G2, float* dx, float* dy, float* dz,
                       float* dux, float* duy, float* duz, float* dw, hipStream_t s) {
  unsigned blocks = (unsigned)std::min<int64_t>(((int64_t)P.nslots + 255) / 256, 16384);
  if (blocks == 0) return;
  hipLaunchKernelGGL((k_backward<O, DIM>), dim3(blocks), dim3(256), 0, s, G, P, G0, G1, G2, dx,
                     dy, dz, dux, duy, duz, dw, err);
}

template <int O, int DIM>
static bool launch_bwd_tile(const KGrid& G, const KPart& P, const pic_bins* b, const float* G0,
                            const float* G1, const float* G2, float* dx, float* dy, float* dz,
                            float* dux, float* duy, float* duz, float* dw, hipStream_t s) {
  const size_t nb = (size_t)b->kb.T[0] * b->kb.T[1] * b->kb.T[2];
  const size_t smem = 3 * sizeof(float) * (size_t)TileWin<O, DIM>::max_size(b->kb) +
                      (nb + 1 + 256) * sizeof(int);   // G windows, particle prefix, scan
  if (smem > b->max_lds) return false;
  // the list count lives in the full sort's scratch counter, the list in its bin array
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, b->kb.ctr + CTR_TOTAL, (int64_t)1);
  hipLaunchKernelGGL((k_backward_tile<O, DIM>), dim3(b->kb.ntiles + TAIL_BLOCKS), dim3(256), smem, s, G,
                     b->kb, P, G0, G1, G2, dx, dy, dz, dux, duy, duz, dw, b->sbin);
  hipLaunchKernelGGL((k_backward_list<O, DIM>), dim3(256), dim3(256), 0, s, G, b->kb, P, G0, G1,
                     G2, dx, dy, dz, dux, duy, duz, dw, b->sbin);
  return true;
}

void backward_launch(const KGrid& G, const KPart& P, const pic_bins* b, const float* G0,
                     const float* G1, const float* G2, float* dx, float* dy, float* dz,
                     float* dux, float* duy, float* duz, float* dw, hipStream_t s) {
  if (b && b->sorted_once) {
    bool ok;
#define BWT(O_, D_) ok = launch_bwd_tile<O_, D_>(G, P, b, G0, G1, G2, dx, dy, dz, dux, duy, duz, dw, s)
    if (G.dim == 3) {
      if (G.order == 1) BWT(1, 3); else if (G.order == 2) BWT(2, 3); else BWT(3, 3);
    } else {
      if (G.order == 1) BWT(1, 2); else if (G.order == 2) BWT(2, 2); else BWT(3, 2);
    }
#undef BWT
    if (ok) return;
  }
  uint32_t* err = b ? b->kb.err : nobins_err_ptr();
#define BWD(O_, D_) launch_bwd<O_, D_>(G, P, err, G0, G1, G2, dx, dy, dz, dux, duy, duz, dw, s)
  if (G.dim == 3) {
    if (G.order == 1) BWD(1, 3); else if (G.order == 2) BWD(2, 3); else BWD(3, 3);
  } else {
    if (G.order == 1) BWD(1, 2); else if (G.order == 2) BWD(2, 2); else BWD(3, 2);
  }
#undef BWD
}
