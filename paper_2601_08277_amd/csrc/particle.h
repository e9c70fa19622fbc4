// Per-particle preparation shared by the deposition and gather kernels: cell and offset
// (Alg. 2, stage 1), current weight w_c = q W v_c (Sec. 4.2.1) and the 1D shape factors.
#pragma once

#include "pic_internal.h"

template <int O, int DIM>
struct PartPrep {
  int cell[3];
  float f[3];
  float amp[3];            // q * W * v_c
  float wn[3][O + 1];      // nodal weights per dimension
  float ws[3][O + 1];      // staggered weights per dimension
  int sn[3], ss[3];        // stencil shifts (nodal, staggered)
};

// Position -> cell + float32 offset (FP64 only here). Returns false (and sets bad) if the
// particle is outside the domain or its position is not finite.
template <int DIM>
__device__ __forceinline__ bool prep_cell(const KGrid& G, double x, double y, double z, int* cell,
                                          float* f, uint32_t& bad) {
  cell[0] = to_cell(x, G.x0[0], G.inv_dx[0], G.n[0], f[0], bad);
  cell[1] = to_cell(y, G.x0[1], G.inv_dx[1], G.n[1], f[1], bad);
  if constexpr (DIM == 3) {
    cell[2] = to_cell(z, G.x0[2], G.inv_dx[2], G.n[2], f[2], bad);
  } else {
    cell[2] = 0;
    f[2] = 0.0f;
  }
  return cell[0] >= 0 && cell[1] >= 0 && cell[2] >= 0;
}

// gamma = sqrt(1 + |u|^2) (c = 1), v = u / gamma, amp_c = q W v_c, in float32.
__device__ __forceinline__ void prep_amp(float q, float ux, float uy, float uz, float w,
                                         float* amp) {
  float ig = 1.0f / sqrtf(1.0f + (ux * ux + uy * uy + uz * uz));
  float qw = q * w * ig;
  amp[0] = qw * ux;
  amp[1] = qw * uy;
  amp[2] = qw * uz;
}

// The same amplitudes with the hardware reciprocal square root (about 1 ulp), times
// `scale`: for staging, where the rsq's error is far below the float32 tolerance.
__device__ __forceinline__ void prep_amp_rsq(float q, float ux, float uy, float uz, float w,
                                             float scale, float* amp) {
  const float ig = __builtin_amdgcn_rsqf(1.0f + (ux * ux + uy * uy + uz * uz));
  const float qw = q * w * ig * scale;
  amp[0] = qw * ux;
  amp[1] = qw * uy;
  amp[2] = qw * uz;
}

template <int O, int DIM>
__device__ __forceinline__ void prep_shapes(PartPrep<O, DIM>& p) {
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    p.sn[d] = shape_w<O, false>(p.f[d], p.wn[d]);
    p.ss[d] = shape_w<O, true>(p.f[d], p.ws[d]);
  }
  if constexpr (DIM == 2) {
    p.sn[2] = p.ss[2] = 0;
#pragma unroll
    for (int k = 0; k <= O; ++k) p.wn[2][k] = p.ws[2][k] = (k == 0) ? 1.0f : 0.0f;
  }
}

// First stencil node (unwrapped) of component c along dimension d.
template <int O, int DIM>
__device__ __forceinline__ int stencil_base(const PartPrep<O, DIM>& p, int c, int d) {
  if (d >= DIM) return 0;
  bool st = (c == d);
  return p.cell[d] + (st ? win_lo(O, true) + p.ss[d] : win_lo(O, false) + p.sn[d]);
}

// Scatter the particle's 3 * (O+1)^DIM contributions through add(c, mx, my, mz, value).
// The component is a template parameter so every weight index is a compile-time constant.
template <int C, int O, int DIM, class Add>
__device__ __forceinline__ void scatter_comp(const PartPrep<O, DIM>& p, Add& add) {
  constexpr int KZ = DIM == 3 ? O + 1 : 1;
  const float* wx = (C == 0) ? p.ws[0] : p.wn[0];
  const float* wy = (C == 1 && DIM >= 2) ? p.ws[1] : p.wn[1];
  const float* wz = (C == 2 && DIM == 3) ? p.ws[2] : p.wn[2];
  const int bx = stencil_base(p, C, 0), by = stencil_base(p, C, 1), bz = stencil_base(p, C, 2);
#pragma unroll
  for (int kz = 0; kz < KZ; ++kz) {
    const float az = p.amp[C] * wz[kz];
#pragma unroll
    for (int ky = 0; ky <= O; ++ky) {
      const float ayz = az * wy[ky];
#pragma unroll
      for (int kx = 0; kx <= O; ++kx) add(C, bx + kx, by + ky, bz + kz, ayz * wx[kx]);
    }
  }
}

template <int O, int DIM, class Add>
__device__ __forceinline__ void scatter_particle(const PartPrep<O, DIM>& p, Add&& add) {
  scatter_comp<0>(p, add);
  scatter_comp<1>(p, add);
  scatter_comp<2>(p, add);
}

// Deposition position of the time-centred current: x + h u / gamma with h = +-dt/2. Only
// the current depends on it (the stored position is not changed), and the shape weights are
// continuous in x, so the offset is formed in float32 (gamma from the hardware reciprocal
// square root, about 1e-7 relative) and added in float64, then wrapped on periodic
// dimensions as in drift_one.
template <int DIM>
__device__ __forceinline__ void midpoint_shift(const KGrid& G, double* pos, float ux, float uy,
                                               float uz, float h) {
  const float hs = h * __builtin_amdgcn_rsqf(1.0f + (ux * ux + uy * uy + uz * uz));
  const float u3[3] = {ux, uy, uz};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    double xn = pos[d] + (double)(hs * u3[d]);
    if (G.per[d]) {
      double t = xn - G.x0[d];
      if (!(t >= 0.0 && t < G.L[d])) t = t - G.L[d] * floor(t / G.L[d]);
      xn = t + G.x0[d];
    }
    pos[d] = xn;
  }
}

// Constant-velocity move in float64 with a fixed operation order (bitwise reproducible):
// s = (ux^2 + uy^2) + uz^2, gamma = sqrt(1 + s), x_d += (u_d / gamma) * dt, then the
// periodic wrap t = x - x0, t - L floor(t / L), + x0. Guard dimensions are not wrapped.
// Every product and sum is rounded on its own: contraction into FMA is switched off here.
template <int DIM>
__device__ __forceinline__ void drift_one(const KGrid& G, double* pos, float ux, float uy,
                                          float uz, double dt) {
#pragma clang fp contract(off)
  const double dux = ux, duy = uy, duz = uz;
  const double s = (dux * dux + duy * duy) + duz * duz;
  const double gam = __builtin_sqrt(1.0 + s);
  const double u3[3] = {dux, duy, duz};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double v = u3[d] / gam;
    double xn = pos[d] + v * dt;
    if (G.per[d]) {
      double t = xn - G.x0[d];
      // t - L floor(t / L); for 0 <= t < L the quotient is below 1, floor gives 0 and t
      // is unchanged, so only the particles that leave the box divide
      if (!(t >= 0.0 && t < G.L[d])) {
        const double fl = floor(t / G.L[d]);
        t = t - G.L[d] * fl;
      }
      xn = t + G.x0[d];
    }
    pos[d] = xn;
  }
}
