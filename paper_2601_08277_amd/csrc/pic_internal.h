// Internal definitions shared by the host API and the gfx950 kernels of libpic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic.h"

#define PIC_MAX_ORDER 3
#define PIC_WAVE 64

// Device error bits (also reported in pic_rebin_stats.error_flags).
enum : uint32_t {
  PIC_EF_DOMAIN = 1u,     // a particle's cell lies outside [0, n)
  PIC_EF_NONFINITE = 2u,  // a position is NaN or infinite
  PIC_EF_CAPACITY = 4u,   // a full sort could not fit the bins into the slots
  PIC_EF_STENCIL = 8u,    // a guard-bounded stencil left the stored nodes
  PIC_EF_MOVE = 16u       // a particle moved a cell or more in one step (charge-conserving)
};

// Device counters kept in the bins object.
enum {
  CTR_NMOV = 0,      // entries in the mover list
  CTR_NOVF = 1,      // movers whose destination bin was full (this rebin)
  CTR_NDROP = 2,     // movers that did not fit the mover list
  CTR_NREB = 3,      // tiles rebuilt (this rebin)
  CTR_NVALID = 4,    // particles held by the bins
  CTR_TOTAL = 5,     // scratch: particles counted by a full sort
  CTR_DESIRED = 6,   // scratch: extra slots wanted by a full sort (low 31 bits)
  CTR_NMOV_LAST = 7, // movers of the last rebin
  CTR_COUNT = 8
};

// Grid as the kernels read it (by value).
struct KGrid {
  int dim, order;
  int n[3];      // cells per dimension (1 for unused dimensions)
  int N[3];      // stored nodes per dimension
  int g[3];      // storage offset of node 0 (ng on guard dimensions, else 0)
  int per[3];    // periodic flag
  double x0[3], inv_dx[3];
  double L[3];   // domain length n * dx (drift wrap)
  float q;
  float inv_dxf[3];
};

// Particle arrays as the kernels read them.
struct KPart {
  double *x, *y, *z;
  float *ux, *uy, *uz, *w;
  int32_t* id;
  int32_t nslots;
};

// Bin tables as the kernels read them.
struct KBins {
  int T[3];          // tile extent in cells
  int nt[3];         // tiles per dimension
  int32_t nbins, ntiles;
  int32_t* off;       // nbins + 1
  int32_t* len;       // nbins
  int32_t* out_flag;  // nbins: 1 if a particle left the bin in this rebin (compaction pending)
  int32_t* ins_cnt;   // nbins
  int32_t* tile_flag; // ntiles
  int32_t* mv_slot;   // max_movers
  int32_t* mv_old;
  int32_t* mv_new;
  int32_t max_movers;
  int32_t* ctr;       // CTR_COUNT
  uint32_t* err;
  float* wscr;        // per-tile stencil windows: ntiles x 3 x wmax floats
  int32_t wmax;       // window floats per component reserved per tile
};

// ---------------------------------------------------------------------------------
// Cell and offset of one coordinate (FP64 on the GPU only for this conversion).
// xi = (x - x0) * inv_dx with both operations rounded separately (contraction is off),
// cell = floor(xi), and xi == n exactly is clamped into n - 1; f = xi - cell (exact), rounded to
// float32. Returns the cell, or -1 outside [0, n) (NaN included; *bad gets the flag).
__device__ __forceinline__ int to_cell(double x, double x0, double inv, int n, float& f,
                                       uint32_t& bad) {
#pragma clang fp contract(off)
  const double xi = (x - x0) * inv;
  double fl = floor(xi);
  fl = xi == (double)n ? (double)(n - 1) : fl;
  const bool fin = __builtin_isfinite(xi);
  const bool in = fl >= 0.0 && fl < (double)n;   // false for NaN
  bad |= !fin ? (uint32_t)PIC_EF_NONFINITE : (!in ? (uint32_t)PIC_EF_DOMAIN : 0u);
  f = (float)(xi - fl);
  return (fin && in) ? (int)(in ? fl : 0.0) : -1;
}

// ---------------------------------------------------------------------------------
// 1D shape factors, Sec. 4.2.1: S = s_x s_y s_z with B-splines of order O, evaluated on
// nodes (nodal) or half-cell positions (staggered component axis). For a particle in
// cell i with offset f, the stencil starts at node  i + win_lo(O, stag) + shift  with
// shift in {0, 1}; the padded window [i + win_lo, i + win_lo + win_w) covers both
// possible starts, so particles of one cell share it.
__host__ __device__ __forceinline__ constexpr int win_lo(int O, bool stag) {
  return O == 1 ? (stag ? -1 : 0) : (O == 2 ? -1 : (stag ? -2 : -1));
}
__host__ __device__ __forceinline__ constexpr int win_w(int O, bool stag) {
  return O == 1 ? (stag ? 3 : 2) : (O == 2 ? (stag ? 3 : 4) : (stag ? 5 : 4));
}

// Weights w[0..O] and the stencil shift. First order: s0 = 1 - d, s1 = d (Sec. 4.2.2);
// second and third order: the cardinal B-spline pieces.
template <int O, bool STAG>
__device__ __forceinline__ int shape_w(float f, float* w) {
  if constexpr (O == 1) {
    int s = 0;
    float t = f;
    if constexpr (STAG) {
      s = f >= 0.5f ? 1 : 0;
      t = s ? f - 0.5f : f + 0.5f;
    }
    w[0] = 1.0f - t;
    w[1] = t;
    return s;
  } else if constexpr (O == 2) {
    int s = 0;
    float g;
    if constexpr (STAG) {
      g = f - 0.5f;
    } else {
      s = f >= 0.5f ? 1 : 0;
      g = s ? f - 1.0f : f;
    }
    float a = 0.5f - g, b = 0.5f + g;
    w[0] = 0.5f * a * a;
    w[1] = 0.75f - g * g;
    w[2] = 0.5f * b * b;
    return s;
  } else {
    int s = 0;
    float t = f;
    if constexpr (STAG) {
      s = f >= 0.5f ? 1 : 0;
      t = s ? f - 0.5f : f + 0.5f;
    }
    const float c6 = 1.0f / 6.0f;
    float u = 1.0f - t, t2 = t * t, t3 = t2 * t;
    w[0] = c6 * u * u * u;
    w[1] = c6 * (4.0f - 6.0f * t2 + 3.0f * t3);
    w[2] = c6 * (1.0f + 3.0f * (t + t2 - t3));
    w[3] = c6 * t3;
    return s;
  }
}

// Third-order weights times 6 (6 w_k), with the same stencil shift as shape_w<3, STAG>:
// (1-t)^3, 4 - 6t^2 + 3t^3, 6 - (the other three), t^3. The per-cell path multiplies the
// amplitude by 1/6^3 once instead of scaling each weight.
template <bool STAG>
__device__ __forceinline__ int shape_w6(float f, float* w) {
  int s = 0;
  float t = f;
  if constexpr (STAG) {
    s = f >= 0.5f ? 1 : 0;
    t = s ? f - 0.5f : f + 0.5f;
  }
  const float u = 1.0f - t, t2 = t * t, t3 = t2 * t;
  w[0] = u * u * u;
  w[1] = 4.0f - 6.0f * t2 + 3.0f * t3;
  w[3] = t3;
  w[2] = 6.0f - w[0] - w[1] - w[3];
  return s;
}

// d/dxi of the weights above (same stencil and shift).
template <int O, bool STAG>
__device__ __forceinline__ int shape_dw(float f, float* dw) {
  if constexpr (O == 1) {
    int s = 0;
    if constexpr (STAG) s = f >= 0.5f ? 1 : 0;
    dw[0] = -1.0f;
    dw[1] = 1.0f;
    return s;
  } else if constexpr (O == 2) {
    int s = 0;
    float g;
    if constexpr (STAG) {
      g = f - 0.5f;
    } else {
      s = f >= 0.5f ? 1 : 0;
      g = s ? f - 1.0f : f;
    }
    dw[0] = g - 0.5f;
    dw[1] = -2.0f * g;
    dw[2] = 0.5f + g;
    return s;
  } else {
    int s = 0;
    float t = f;
    if constexpr (STAG) {
      s = f >= 0.5f ? 1 : 0;
      t = s ? f - 0.5f : f + 0.5f;
    }
    float u = 1.0f - t;
    dw[0] = -0.5f * u * u;
    dw[1] = t * (1.5f * t - 2.0f);
    dw[2] = 0.5f + t - 1.5f * t * t;
    dw[3] = 0.5f * t * t;
    return s;
  }
}

// Storage index along one dimension of node m (periodic wrap or guard offset).
// Returns -1 if a guard-bounded node falls outside the stored range.
__device__ __forceinline__ int store_idx(const KGrid& G, int d, int m) {
  if (G.per[d]) {
    if (m < 0) m += G.n[d];
    else if (m >= G.n[d]) m -= G.n[d];
    return m;
  }
  m += G.g[d];
  return (m >= 0 && m < G.N[d]) ? m : -1;
}

// ---------------------------------------------------------------------------------
// Bins: tiles x fastest, cells x fastest inside a tile (edge tiles may be smaller).
struct TileBox {
  int c0[3];   // first cell
  int e[3];    // extent in cells
  int32_t b0;  // first bin
  int32_t nb;  // bins (cells) in the tile
};

// Tile of workgroup b in a one-workgroup-per-tile launch of n workgroups. Workgroups go to
// the 8 XCDs in turn (b mod 8), so XCD j is given the j-th contiguous eighth of the tiles:
// neighbouring tiles, which read each other's window halos, then share one L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  constexpr int X = 8;
  const int q = n / X, r = n % X;
  const int j = b % X, k = b / X;
  return j * q + min(j, r) + k;
}

__host__ __device__ __forceinline__ TileBox tile_box(const int n[3], const int T[3],
                                                     const int nt[3], int t) {
  TileBox tb;
  int tx = t % nt[0], ty = (t / nt[0]) % nt[1], tz = t / (nt[0] * nt[1]);
  tb.c0[0] = tx * T[0];
  tb.c0[1] = ty * T[1];
  tb.c0[2] = tz * T[2];
  tb.e[0] = min(T[0], n[0] - tb.c0[0]);
  tb.e[1] = min(T[1], n[1] - tb.c0[1]);
  tb.e[2] = min(T[2], n[2] - tb.c0[2]);
  tb.b0 = (int32_t)((int64_t)tb.c0[2] * n[0] * n[1] + (int64_t)tb.c0[1] * n[0] * tb.e[2] +
                    (int64_t)tb.c0[0] * tb.e[1] * tb.e[2]);
  tb.nb = tb.e[0] * tb.e[1] * tb.e[2];
  return tb;
}

__host__ __device__ __forceinline__ int32_t bin_of_cell(const int n[3], const int T[3], int i,
                                                        int j, int k) {
  int tx = i / T[0], ty = j / T[1], tz = k / T[2];
  int c0x = tx * T[0], c0y = ty * T[1], c0z = tz * T[2];
  int ez = min(T[2], n[2] - c0z), ey = min(T[1], n[1] - c0y), ex = min(T[0], n[0] - c0x);
  int64_t b0 = (int64_t)c0z * n[0] * n[1] + (int64_t)c0y * n[0] * ez + (int64_t)c0x * ey * ez;
  return (int32_t)(b0 + (i - c0x) + ex * ((j - c0y) + ey * (k - c0z)));
}

__host__ __device__ __forceinline__ int tile_of_cell(const int T[3], const int nt[3], int i,
                                                     int j, int k) {
  return (i / T[0]) + nt[0] * ((j / T[1]) + nt[1] * (k / T[2]));
}

// Wave-aggregated append to a device list: one atomic per wave. Every lane of the wave
// must call it. Returns the slot for lanes with pred, -1 otherwise.
__device__ __forceinline__ int wave_append(bool pred, int32_t* counter) {
  unsigned long long m = __ballot(pred);
  if (m == 0ull) return -1;
  int lane = __lane_id();
  int leader = __ffsll((long long)m) - 1;
  int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                       __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, (int)__popcll(m));
  base = __shfl(base, leader);
  return pred ? base + rank : -1;
}

// ---------------------------------------------------------------------------------
// Host-side launch helpers implemented in the .hip files.
struct pic_bins_impl;
void launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
void launch_zero_j3(float* a, float* b, float* c, int64_t n, hipStream_t s,
                    int32_t* ctr = nullptr);
