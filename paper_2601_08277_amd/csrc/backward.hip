// Adjoint of the deposition: for L = sum_c <G_c, J_c> every particle gathers G with the
// same shape factors (recomputed, not stored) and their derivatives. The gather is the
// field-interpolation pattern of Sec. 3.1 run backwards through Eq. 1:
//   g_c      = sum_nodes G_c * S_c                      (S_c = s_x s_y s_z, staggered on c)
//   h_{c,d}  = sum_nodes G_c * dS_c/dxi_d
//   dL/dw    = q * sum_c v_c g_c
//   dL/du_b  = q W (g_b / gamma - u_b (sum_c u_c g_c) / gamma^3)
//   dL/dx_d  = q W sum_c v_c h_{c,d} * inv_dx_d
#include <algorithm>

#include "particle.h"
#include "pic_host.h"

uint32_t* nobins_err_ptr();

template <int O, int DIM>
__global__ __launch_bounds__(256) void k_backward(KGrid G, KPart P, const float* __restrict__ G0,
                                                  const float* __restrict__ G1,
                                                  const float* __restrict__ G2,
                                                  float* __restrict__ dx, float* __restrict__ dy,
                                                  float* __restrict__ dz, float* __restrict__ dux,
                                                  float* __restrict__ duy, float* __restrict__ duz,
                                                  float* __restrict__ dw, uint32_t* err) {
  constexpr int KZ = DIM == 3 ? O + 1 : 1;
  const float* Gs[3] = {G0, G1, G2};
  uint32_t bad = 0;
  const int stride = gridDim.x * blockDim.x;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < P.nslots; s += stride) {
    float r_dx[3] = {0.f, 0.f, 0.f}, r_du[3] = {0.f, 0.f, 0.f}, r_dw = 0.f;
    int cell[3];
    float f[3];
    bool ok = P.id[s] != PIC_INVALID_ID &&
              prep_cell<DIM>(G, P.x[s], P.y[s], DIM == 3 ? P.z[s] : 0.0, cell, f, bad);
    if (ok) {
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
          int iz = DIM == 3 ? store_idx(G, 2, bse[2] + kz) : 0;
#pragma unroll
          for (int ky = 0; ky <= O; ++ky) {
            int iy = store_idx(G, 1, bse[1] + ky);
            float sx = 0.f, dsx = 0.f;
#pragma unroll
            for (int kx = 0; kx <= O; ++kx) {
              int ix = store_idx(G, 0, bse[0] + kx);
              float gv = 0.f;
              if ((ix | iy | iz) >= 0) gv = Gs[c][((int64_t)iz * G.N[1] + iy) * G.N[0] + ix];
              else if (W[0][kx] * W[1][ky] * W[2][kz] != 0.f) bad |= PIC_EF_STENCIL;
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
      r_dw = G.q * (v[0] * gsum[0] + v[1] * gsum[1] + v[2] * gsum[2]);
      const float ug = u[0] * gsum[0] + u[1] * gsum[1] + u[2] * gsum[2];
      const float ig3 = ig * ig * ig;
#pragma unroll
      for (int b = 0; b < 3; ++b) r_du[b] = wq * (gsum[b] * ig - u[b] * ug * ig3);
#pragma unroll
      for (int d = 0; d < DIM; ++d)
        r_dx[d] = wq * (v[0] * h[0][d] + v[1] * h[1][d] + v[2] * h[2][d]) * G.inv_dxf[d];
    }
    dx[s] = r_dx[0];
    dy[s] = r_dx[1];
    if (DIM == 3) dz[s] = r_dx[2];
    dux[s] = r_du[0];
    duy[s] = r_du[1];
    duz[s] = r_du[2];
    if (dw) dw[s] = r_dw;
  }
  if (bad) atomicOr(err, bad);
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

void backward_launch(const KGrid& G, const KPart& P, const pic_bins* b, const float* G0,
                     const float* G1, const float* G2, float* dx, float* dy, float* dz,
                     float* dux, float* duy, float* duz, float* dw, hipStream_t s) {
  uint32_t* err = b ? b->kb.err : nobins_err_ptr();
#define BWD(O_, D_) launch_bwd<O_, D_>(G, P, err, G0, G1, G2, dx, dy, dz, dux, duy, duz, dw, s)
  if (G.dim == 3) {
    if (G.order == 1) BWD(1, 3); else if (G.order == 2) BWD(2, 3); else BWD(3, 3);
  } else {
    if (G.order == 1) BWD(1, 2); else if (G.order == 2) BWD(2, 2); else BWD(3, 2);
  }
#undef BWD
}
