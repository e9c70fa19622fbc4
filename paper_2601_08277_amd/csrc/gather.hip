// Field gather: E and B interpolated to the particles with the deposition's shape factors
// (the field-interpolation half of the PIC cycle, Sec. 3.1; the forward of the adjoint's
// gather). E_c sits on the edge along its own axis (as J_c); B_c on the face normal to c,
// half a cell along the two other axes.
//
// Tiled like the adjoint: one workgroup per particle tile loads the tile's stencil window
// of all six components into LDS, then its particles gather from LDS. Particles whose cell
// is outside their tile are listed and gathered from global memory by k_gather_list.
#include <algorithm>
#include <cmath>

#include "deposit_common.h"
#include "tile_particles.h"

uint32_t* nobins_err_ptr();

// The 1D weights and first nodes of one dimension, nodal and half-cell staggered: the six
// field components use only these six vectors, so they are formed once per particle.
template <int O>
struct GatherW {
  float w[2][O + 1];   // [staggered][k]
  int b[2];
};

template <int O, int DIM>
__device__ __forceinline__ void gather_weights(const int* cell, const float* f, GatherW<O>* gw) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d < DIM) {
      gw[d].b[0] = cell[d] + win_lo(O, false) + shape_w<O, false>(f[d], gw[d].w[0]);
      gw[d].b[1] = cell[d] + win_lo(O, true) + shape_w<O, true>(f[d], gw[d].w[1]);
    } else {          // 2D: one node along z with weight 1
#pragma unroll
      for (int k = 0; k <= O; ++k) gw[d].w[0][k] = gw[d].w[1][k] = k == 0 ? 1.0f : 0.0f;
      gw[d].b[0] = gw[d].b[1] = 0;
    }
  }
}

// Sum over the stencil of field component c at the particle, with per-dimension
// staggering SX, SY, SZ.
template <int O, int DIM, bool SX, bool SY, bool SZ, class Fetch>
__device__ __forceinline__ float gather_one(const GatherW<O>* gw, int c, Fetch&& fetch) {
  const float* wx = gw[0].w[SX];
  const float* wy = gw[1].w[SY];
  const float* wz = gw[2].w[SZ];
  const int bx = gw[0].b[SX], by = gw[1].b[SY], bz = gw[2].b[SZ];
  float acc = 0.0f;
#pragma unroll
  for (int kz = 0; kz < (DIM == 3 ? O + 1 : 1); ++kz) {
#pragma unroll
    for (int ky = 0; ky <= O; ++ky) {
      float sx = 0.0f;
#pragma unroll
      for (int kx = 0; kx <= O; ++kx)
        sx += wx[kx] * fetch(c, bx + kx, by + ky, bz + kz, wx[kx] * wy[ky] * wz[kz]);
      acc += wz[kz] * wy[ky] * sx;
    }
  }
  return acc;
}

// The six gathered components of one particle; out[0..2] = E, out[3..5] = B.
template <int O, int DIM, class Fetch>
__device__ __forceinline__ void gather_particle(const int* cell, const float* f, Fetch&& fetch,
                                                float* out) {
  constexpr bool Z3 = DIM == 3;
  GatherW<O> gw[3];
  gather_weights<O, DIM>(cell, f, gw);
  out[0] = gather_one<O, DIM, true, false, false>(gw, 0, fetch);
  out[1] = gather_one<O, DIM, false, true, false>(gw, 1, fetch);
  out[2] = gather_one<O, DIM, false, false, Z3>(gw, 2, fetch);
  out[3] = gather_one<O, DIM, false, true, Z3>(gw, 3, fetch);
  out[4] = gather_one<O, DIM, true, false, Z3>(gw, 4, fetch);
  out[5] = gather_one<O, DIM, true, true, false>(gw, 5, fetch);
}

struct GatherOut {
  float* p[6];
};

struct FieldFetch {
  const KGrid& G;
  const float* const* F;
  uint32_t& bad;
  __device__ __forceinline__ float operator()(int c, int mx, int my, int mz, float w) const {
    const int ix = store_idx(G, 0, mx), iy = store_idx(G, 1, my);
    const int iz = G.dim == 3 ? store_idx(G, 2, mz) : 0;
    if ((ix | iy | iz) >= 0) return F[c][((int64_t)iz * G.N[1] + iy) * G.N[0] + ix];
    if (w != 0.f) bad |= PIC_EF_STENCIL;
    return 0.f;
  }
};

struct FieldPtrs {
  const float* f[6];
};

// Weight k of a stencil vector by select, for a lane-dependent k (an indexed register
// array would go to scratch memory).
template <int O>
__device__ __forceinline__ float gw_pick(const float* w, int k) {
  float v = w[0];
#pragma unroll
  for (int i = 1; i <= O; ++i) v = k == i ? w[i] : v;
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = PIC_WAVE / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

template <int O, int DIM, bool SX, bool SY, bool SZ>
__device__ __forceinline__ float wave_gather_one(const GatherW<O>* gw, int c, int kx, int ky,
                                                 int kz, bool act, const FieldFetch& ff) {
  float t = 0.0f;
  if (act) {
    const float w = gw_pick<O>(gw[0].w[SX], kx) * gw_pick<O>(gw[1].w[SY], ky) *
                    gw_pick<O>(gw[2].w[SZ], kz);
    t = w * ff(c, gw[0].b[SX] + kx, gw[1].b[SY] + ky, gw[2].b[SZ] + kz, w);
  }
  return wave_sum(t);
}

// The six components of one particle gathered by a whole wave, lanes = stencil nodes (for
// the few particles outside their tile's window: their nodes are read from global memory
// by 64 lanes at once instead of one after another). Every lane returns the sums.
template <int O, int DIM>
__device__ __forceinline__ void wave_gather(const int* cell, const float* f, const FieldFetch& ff,
                                            float* v) {
  constexpr int NS = (O + 1) * (O + 1) * (DIM == 3 ? O + 1 : 1);
  constexpr bool Z3 = DIM == 3;
  GatherW<O> gw[3];
  gather_weights<O, DIM>(cell, f, gw);
  const int lane = threadIdx.x % PIC_WAVE;
  const bool act = lane < NS;
  const int kx = lane % (O + 1), ky = (lane / (O + 1)) % (O + 1);
  const int kz = DIM == 3 ? lane / ((O + 1) * (O + 1)) : 0;
  v[0] = wave_gather_one<O, DIM, true, false, false>(gw, 0, kx, ky, kz, act, ff);
  v[1] = wave_gather_one<O, DIM, false, true, false>(gw, 1, kx, ky, kz, act, ff);
  v[2] = wave_gather_one<O, DIM, false, false, Z3>(gw, 2, kx, ky, kz, act, ff);
  v[3] = wave_gather_one<O, DIM, false, true, Z3>(gw, 3, kx, ky, kz, act, ff);
  v[4] = wave_gather_one<O, DIM, true, false, Z3>(gw, 4, kx, ky, kz, act, ff);
  v[5] = wave_gather_one<O, DIM, true, true, false>(gw, 5, kx, ky, kz, act, ff);
}

__device__ __forceinline__ void gather_write(const GatherOut& o, int s, const float* v) {
#pragma unroll
  for (int c = 0; c < 6; ++c) o.p[c][s] = v[c];
}

// LDS of the gather and push tile kernels: six field windows, the tile's particle prefix
// (one int per bin plus one) and the scan's 256 ints.
template <int O, int DIM>
static size_t tile_kernel_smem(const KBins& kb) {
  const size_t nb = (size_t)kb.T[0] * kb.T[1] * kb.T[2];
  return 6 * sizeof(float) * (size_t)TileWin<O, DIM>::max_size(kb) + (nb + 1 + 256) * sizeof(int);
}

// Particle-parallel gather from global memory (no bins).
template <int O, int DIM>
__global__ __launch_bounds__(256) void k_gather(KGrid G, KPart P, FieldPtrs F, GatherOut o,
                                                uint32_t* err) {
  uint32_t bad = 0;
  const FieldFetch ff{G, F.f, bad};
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < P.nslots; s += gridDim.x * blockDim.x) {
    int cell[3];
    float f[3];
    float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (P.id[s] != PIC_INVALID_ID &&
        prep_cell<DIM>(G, P.x[s], P.y[s], DIM == 3 ? P.z[s] : 0.0, cell, f, bad))
      gather_particle<O, DIM>(cell, f, ff, v);
    gather_write(o, s, v);
  }
  if (bad) atomicOr(err, bad);
}

template <int O, int DIM>
__global__ __launch_bounds__(256) void k_gather_tile(KGrid G, KBins B, KPart P, FieldPtrs F,
                                                     GatherOut o, int32_t* __restrict__ list) {
  extern __shared__ __align__(16) float sF[];
  uint32_t bad = 0;
  if (blockIdx.x >= (unsigned)B.ntiles) {
    const float z[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int stride = TAIL_BLOCKS * blockDim.x;
    for (int s = B.off[B.nbins] + (blockIdx.x - B.ntiles) * blockDim.x + threadIdx.x;
         s < P.nslots; s += stride)
      gather_write(o, s, z);
    return;
  }
  const TileBox tb = tile_box(G.n, B.T, B.nt, blockIdx.x);
  const TileWin<O, DIM> tw(tb);
  for (int i = threadIdx.x; i < 6 * tw.size; i += blockDim.x) {
    const int c = i / tw.size;
    const int r = i - c * tw.size;
    const int W01 = tw.W[0] * tw.W[1];
    const int wz = r / W01, wy = (r - wz * W01) / tw.W[0], wx = r - wz * W01 - wy * tw.W[0];
    const int ix = store_idx(G, 0, tw.o[0] + wx), iy = store_idx(G, 1, tw.o[1] + wy);
    const int iz = DIM == 3 ? store_idx(G, 2, tw.o[2] + wz) : 0;
    sF[i] = (ix | iy | iz) >= 0 ? F.f[c][((int64_t)iz * G.N[1] + iy) * G.N[0] + ix] : 0.f;
  }
  __syncthreads();
  auto lf = [&](int c, int mx, int my, int mz, float) -> float {
    return sF[c * tw.size + ((mz - tw.o[2]) * tw.W[1] + (my - tw.o[1])) * tw.W[0] + (mx - tw.o[0])];
  };
  int* pre = (int*)(sF + 6 * tw.size);
  const int nval = tile_valid_prefix(B, tb, pre, pre + tb.nb + 1);
  // gap slots get zeros
  const int S0 = B.off[tb.b0], S1 = B.off[tb.b0 + tb.nb];
  const float z[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int s = S0 + threadIdx.x; s < S1; s += blockDim.x)
    if (P.id[s] == PIC_INVALID_ID) gather_write(o, s, z);
  for (int base = 0; base < nval; base += blockDim.x) {
    const int j = base + threadIdx.x;
    const int s = j < nval ? tile_valid_slot(B, tb, pre, j) : 0;
    int cell[3];
    float f[3];
    const bool ok = j < nval &&
                    prep_cell<DIM>(G, P.x[s], P.y[s], DIM == 3 ? P.z[s] : 0.0, cell, f, bad);
    const bool local = ok && tw.fits_cell(cell);
    float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (local) gather_particle<O, DIM>(cell, f, lf, v);
    if (j < nval && (local || !ok)) gather_write(o, s, v);
    const int e = wave_append(ok && !local, &B.ctr[CTR_TOTAL]);
    if (e >= 0) list[e] = s;
  }
  if (bad) atomicOr(B.err, bad);
}

template <int O, int DIM>
__global__ __launch_bounds__(256) void k_gather_list(KGrid G, KBins B, KPart P, FieldPtrs F,
                                                     GatherOut o,
                                                     const int32_t* __restrict__ list) {
  uint32_t bad = 0;
  const FieldFetch ff{G, F.f, bad};
  const int n = B.ctr[CTR_TOTAL];
  const int lane = threadIdx.x % PIC_WAVE;
  const int nw = gridDim.x * (blockDim.x / PIC_WAVE);
  // one listed particle per wave (wave-uniform loop)
  for (int e = blockIdx.x * (blockDim.x / PIC_WAVE) + threadIdx.x / PIC_WAVE; e < n; e += nw) {
    const int s = list[e];
    int cell[3];
    float f[3];
    float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (prep_cell<DIM>(G, P.x[s], P.y[s], DIM == 3 ? P.z[s] : 0.0, cell, f, bad))
      wave_gather<O, DIM>(cell, f, ff, v);
    if (lane == 0) gather_write(o, s, v);
  }
  if (bad) atomicOr(B.err, bad);
}

template <int O, int DIM>
static void launch_gather(const KGrid& G, const KPart& P, pic_bins* b, const FieldPtrs& F,
                          const GatherOut& o, hipStream_t s) {
  const size_t smem = b ? tile_kernel_smem<O, DIM>(b->kb) : 0;
  if (b && b->sorted_once && smem <= b->max_lds) {
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, b->kb.ctr + CTR_TOTAL, (int64_t)1);
    hipLaunchKernelGGL((k_gather_tile<O, DIM>), dim3(b->kb.ntiles + TAIL_BLOCKS), dim3(256), smem, s, G,
                       b->kb, P, F, o, b->sbin);
    hipLaunchKernelGGL((k_gather_list<O, DIM>), dim3(256), dim3(256), 0, s, G, b->kb, P, F, o,
                       b->sbin);
    return;
  }
  const unsigned blocks = (unsigned)std::min<int64_t>(((int64_t)P.nslots + 255) / 256, 16384);
  if (blocks == 0) return;
  hipLaunchKernelGGL((k_gather<O, DIM>), dim3(blocks), dim3(256), 0, s, G, P, F, o,
                     b ? b->kb.err : nobins_err_ptr());
}

extern "C" pic_status pic_gather_fields(const pic_grid* grid, const pic_particles* p,
                                        pic_bins* b, const float* Ex, const float* Ey,
                                        const float* Ez, const float* Bx, const float* By,
                                        const float* Bz, float* ex, float* ey, float* ez,
                                        float* bx, float* by, float* bz, hipStream_t stream) {
  pic_status st = validate_grid(grid);
  if (st != PIC_OK) return st;
  if ((st = validate_particles(p, grid->dim)) != PIC_OK) return st;
  if (!Ex || !Ey || !Ez || !Bx || !By || !Bz || !ex || !ey || !ez || !bx || !by || !bz)
    return set_error(PIC_ERR_INVALID_ARG, "field and output pointers must not be NULL");
  if (b) {
    if (!same_grid(*grid, b->grid)) return set_error(PIC_ERR_INVALID_ARG, "grid differs from the bins' grid");
    if (p->nslots != b->nslots) return set_error(PIC_ERR_INVALID_ARG, "nslots differs from the bins' nslots");
  }
  const KGrid G = make_kgrid(*grid);
  const KPart P = make_kpart(*p);
  const FieldPtrs F{{Ex, Ey, Ez, Bx, By, Bz}};
  const GatherOut o{{ex, ey, ez, bx, by, bz}};
#define GA(O_, D_) launch_gather<O_, D_>(G, P, b, F, o, stream)
  if (G.dim == 3) {
    if (G.order == 1) GA(1, 3); else if (G.order == 2) GA(2, 3); else GA(3, 3);
  } else {
    if (G.order == 1) GA(1, 2); else if (G.order == 2) GA(2, 2); else GA(3, 2);
  }
#undef GA
  return check_hip(hipGetLastError(), "pic_gather_fields launch");
}

// ---------------------------------------------------------------------------------------
// Particle push: the gather above followed by the relativistic Boris rotation (c = 1,
// h = qm dt / 2) and the move, one pass over the particles. With u- = u + h E,
// t = h B / gamma(u-), s = 2 t / (1 + |t|^2): u+ = u- + (u- + u- x t) x s, u <- u+ + h E,
// all in float32 like the stored momenta; then x moves with the new u exactly as
// drift_one does (the position update stays in float64, like the positions).

__device__ __forceinline__ void cross3(const float* a, const float* b, float* r) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}

template <int DIM>
__device__ __forceinline__ void boris_move(const KGrid& G, const KPart& P, int s, const float* v,
                                           float h, double dt) {
  // every load before the first store: the arrays may alias, which would keep a later
  // load behind an earlier store
  double pos[3] = {P.x[s], P.y[s], DIM == 3 ? P.z[s] : 0.0};
  const float um[3] = {P.ux[s] + h * v[0], P.uy[s] + h * v[1], P.uz[s] + h * v[2]};
  const float ig = 1.0f / __builtin_sqrtf(1.0f + ((um[0] * um[0] + um[1] * um[1]) + um[2] * um[2]));
  const float t[3] = {h * v[3] * ig, h * v[4] * ig, h * v[5] * ig};
  const float k = 2.0f / (1.0f + ((t[0] * t[0] + t[1] * t[1]) + t[2] * t[2]));
  const float sv[3] = {k * t[0], k * t[1], k * t[2]};
  float c[3], up[3];
  cross3(um, t, c);
#pragma unroll
  for (int d = 0; d < 3; ++d) up[d] = um[d] + c[d];
  cross3(up, sv, c);
  const float un[3] = {um[0] + c[0] + h * v[0], um[1] + c[1] + h * v[1],
                       um[2] + c[2] + h * v[2]};
  P.ux[s] = un[0];
  P.uy[s] = un[1];
  P.uz[s] = un[2];
  drift_one<DIM>(G, pos, un[0], un[1], un[2], dt);
  P.x[s] = pos[0];
  P.y[s] = pos[1];
  if (DIM == 3) P.z[s] = pos[2];
}

// Particle-parallel push from global memory (no bins).
template <int O, int DIM>
__global__ __launch_bounds__(256) void k_push(KGrid G, KPart P, FieldPtrs F, float h, double dt,
                                              uint32_t* err) {
  uint32_t bad = 0;
  const FieldFetch ff{G, F.f, bad};
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < P.nslots; s += gridDim.x * blockDim.x) {
    int cell[3];
    float f[3];
    if (P.id[s] == PIC_INVALID_ID ||
        !prep_cell<DIM>(G, P.x[s], P.y[s], DIM == 3 ? P.z[s] : 0.0, cell, f, bad))
      continue;
    float v[6];
    gather_particle<O, DIM>(cell, f, ff, v);
    boris_move<DIM>(G, P, s, v, h, dt);
  }
  if (bad) atomicOr(err, bad);
}

// One workgroup per tile: the six field windows into LDS, then every particle of the tile
// whose stencil lies in the window is pushed from LDS. Particles outside their tile's
// window are listed for k_push_list. Slots past the last bin are gaps (the bins hold every
// valid particle) and are not visited.
template <int O, int DIM>
__global__ __launch_bounds__(256) void k_push_tile(KGrid G, KBins B, KPart P, FieldPtrs F,
                                                   float h, double dt,
                                                   int32_t* __restrict__ list) {
  extern __shared__ __align__(16) float sF[];
  uint32_t bad = 0;
  const TileBox tb = tile_box(G.n, B.T, B.nt, blockIdx.x);
  const TileWin<O, DIM> tw(tb);
  const int W01 = tw.W[0] * tw.W[1];
  for (int i = threadIdx.x; i < 6 * tw.size; i += blockDim.x) {
    const int c = i / tw.size;
    const int r = i - c * tw.size;
    const int wz = r / W01, wy = (r - wz * W01) / tw.W[0], wx = r - wz * W01 - wy * tw.W[0];
    const int ix = store_idx(G, 0, tw.o[0] + wx), iy = store_idx(G, 1, tw.o[1] + wy);
    const int iz = DIM == 3 ? store_idx(G, 2, tw.o[2] + wz) : 0;
    sF[i] = (ix | iy | iz) >= 0 ? F.f[c][((int64_t)iz * G.N[1] + iy) * G.N[0] + ix] : 0.f;
  }
  __syncthreads();
  auto lf = [&](int c, int mx, int my, int mz, float) -> float {
    return sF[c * tw.size + ((mz - tw.o[2]) * tw.W[1] + (my - tw.o[1])) * tw.W[0] + (mx - tw.o[0])];
  };
  int* pre = (int*)(sF + 6 * tw.size);
  const int nval = tile_valid_prefix(B, tb, pre, pre + tb.nb + 1);
  for (int base = 0; base < nval; base += blockDim.x) {
    const int j = base + threadIdx.x;
    const int s = j < nval ? tile_valid_slot(B, tb, pre, j) : 0;
    int cell[3];
    float f[3];
    const bool ok = j < nval &&
                    prep_cell<DIM>(G, P.x[s], P.y[s], DIM == 3 ? P.z[s] : 0.0, cell, f, bad);
    const bool local = ok && tw.fits_cell(cell);
    if (local) {
      float v[6];
      gather_particle<O, DIM>(cell, f, lf, v);
      boris_move<DIM>(G, P, s, v, h, dt);
    }
    const int e = wave_append(ok && !local, &B.ctr[CTR_TOTAL]);
    if (e >= 0) list[e] = s;
  }
  if (bad) atomicOr(B.err, bad);
}

template <int O, int DIM>
__global__ __launch_bounds__(256) void k_push_list(KGrid G, KBins B, KPart P, FieldPtrs F,
                                                   float h, double dt,
                                                   const int32_t* __restrict__ list) {
  uint32_t bad = 0;
  const FieldFetch ff{G, F.f, bad};
  const int n = B.ctr[CTR_TOTAL];
  const int lane = threadIdx.x % PIC_WAVE;
  const int nw = gridDim.x * (blockDim.x / PIC_WAVE);
  // one listed particle per wave (wave-uniform loop); lane 0 pushes it
  for (int e = blockIdx.x * (blockDim.x / PIC_WAVE) + threadIdx.x / PIC_WAVE; e < n; e += nw) {
    const int s = list[e];
    int cell[3];
    float f[3];
    if (!prep_cell<DIM>(G, P.x[s], P.y[s], DIM == 3 ? P.z[s] : 0.0, cell, f, bad)) continue;
    float v[6];
    wave_gather<O, DIM>(cell, f, ff, v);
    if (lane == 0) boris_move<DIM>(G, P, s, v, h, dt);
  }
  if (bad) atomicOr(B.err, bad);
}

template <int O, int DIM>
static void launch_push(const KGrid& G, const KPart& P, pic_bins* b, const FieldPtrs& F,
                        float h, double dt, hipStream_t s) {
  const size_t smem = b ? tile_kernel_smem<O, DIM>(b->kb) : 0;
  if (b && b->sorted_once && smem <= b->max_lds) {
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, b->kb.ctr + CTR_TOTAL, (int64_t)1);
    hipLaunchKernelGGL((k_push_tile<O, DIM>), dim3(b->kb.ntiles), dim3(256), smem, s, G,
                       b->kb, P, F, h, dt, b->sbin);
    hipLaunchKernelGGL((k_push_list<O, DIM>), dim3(256), dim3(256), 0, s, G, b->kb, P, F, h, dt,
                       b->sbin);
    return;
  }
  const unsigned blocks = (unsigned)std::min<int64_t>(((int64_t)P.nslots + 255) / 256, 16384);
  if (blocks == 0) return;
  hipLaunchKernelGGL((k_push<O, DIM>), dim3(blocks), dim3(256), 0, s, G, P, F, h, dt,
                     b ? b->kb.err : nobins_err_ptr());
}

extern "C" pic_status pic_push(const pic_grid* grid, pic_particles* p, pic_bins* b,
                               const float* Ex, const float* Ey, const float* Ez,
                               const float* Bx, const float* By, const float* Bz, double qm,
                               double dt, unsigned flags, hipStream_t stream) {
  pic_status st = validate_grid(grid);
  if (st != PIC_OK) return st;
  if ((st = validate_particles(p, grid->dim)) != PIC_OK) return st;
  if (!Ex || !Ey || !Ez || !Bx || !By || !Bz)
    return set_error(PIC_ERR_INVALID_ARG, "field pointers must not be NULL");
  if (!std::isfinite(qm) || !std::isfinite(dt))
    return set_error(PIC_ERR_INVALID_ARG, "qm and dt must be finite");
  if (flags != 0) return set_error(PIC_ERR_INVALID_ARG, "pic_push takes no flags");
  if (b) {
    if (!same_grid(*grid, b->grid)) return set_error(PIC_ERR_INVALID_ARG, "grid differs from the bins' grid");
    if (p->nslots != b->nslots) return set_error(PIC_ERR_INVALID_ARG, "nslots differs from the bins' nslots");
  }
  const KGrid G = make_kgrid(*grid);
  const KPart P = make_kpart(*p);
  const FieldPtrs F{{Ex, Ey, Ez, Bx, By, Bz}};
  const float h = (float)(0.5 * qm * dt);
#define PU(O_, D_) launch_push<O_, D_>(G, P, b, F, h, dt, stream)
  if (G.dim == 3) {
    if (G.order == 1) PU(1, 3); else if (G.order == 2) PU(2, 3); else PU(3, 3);
  } else {
    if (G.order == 1) PU(1, 2); else if (G.order == 2) PU(2, 2); else PU(3, 2);
  }
#undef PU
  if (b) b->movers_fresh = false;
  return check_hip(hipGetLastError(), "pic_push launch");
}
