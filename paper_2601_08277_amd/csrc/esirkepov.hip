// Charge-conserving current deposition (Esirkepov's density decomposition).
//
// The paper deposits the direct current of Eq. 1 and lists charge-conserving schemes as
// unsupported (Sec. 7). For a particle moving from grid coordinate xi0 to xi1 within one
// step (less than a cell per dimension), with 1D nodal B-spline weights S0, S1 on a common
// box of O+2 nodes per dimension, DS = S1 - S0 and M = (S0 + S1)/2, the published
// decomposition (Esirkepov, Comput. Phys. Commun. 135 (2001) 144) gives in 3D
//
//   Jx(i+1/2, j, k) = A_x(i) * (M_y(j) M_z(k) + DS_y(j) DS_z(k) / 12),
//   A_x(i) = -q W dx/dt * sum_{i' <= i} DS_x(i'),
//
// since S0y S0z + DSy S0z/2 + S0y DSz/2 + DSy DSz/3 = My Mz + DSy DSz/12 (the same holds
// for y and z by exchange). In 2D, Jx = A_x(i) M_y(j), Jy likewise, and the out-of-plane
// Jz = q W v_z (Mx My + DSx DSy / 12). So every component is a sum of at most two outer
// products of short per-particle vectors, which is how the kernels evaluate it.
//
// The weights are formed in float64: DS is a difference of two weights close to each
// other for small moves, and float32 would lose most of its digits there. The factor
// vectors are then rounded to float32 and the outer products accumulated in float32.
//
// Tiled path (bins filled by pic_rebin): one workgroup per tile; wave 3 prepares 64
// particles at a time (one per lane, float64) into a double-buffered LDS record list;
// waves 0-2 each own one J component of an LDS window covering the tile plus a margin of
// ML cells and add each particle's box with lanes = box nodes (plain read-add-write: one
// particle per instruction touches distinct nodes, and one wave owns each component).
// Particles whose box does not fit the window are added with global atomics. The window
// is then added to J with one global atomic per non-zero entry.
#include <algorithm>
#include <cmath>

#include "deposit_common.h"

uint32_t* nobins_err_ptr();

namespace {

constexpr int ESK_WAVES = 4;
constexpr int ESK_CHUNK = PIC_WAVE;

template <int O>
constexpr int esk_margin() {
  return (O + 1) / 2 + 2;
}

// record: [0] window base (int bits), [1] q W v_z (2D), then per dimension M[O+2],
// DS[O+2], A[O+1]; odd length, so that 64 lanes writing one record each hit distinct banks
template <int O, int DIM>
constexpr int esk_rec() {
  return (2 + DIM * (3 * O + 5)) | 1;
}

// Box extent of component C along dimension D: O+1 faces along the component's own axis,
// O+2 nodes across it; in 2D the out-of-plane component has O+2 nodes along x and y.
template <int O, int DIM, int C, int D>
constexpr int esk_ext() {
  return D < DIM ? (D == C ? O + 1 : O + 2) : 1;
}

// Nodal B-spline weights of order O at grid coordinate xi (float64): the O+1 non-zero
// weights, first at node `start`. Order 1: start = floor(xi), weights 1-f, f. Order 2:
// m = floor(xi + 1/2), d = xi - m, start = m - 1, weights (1/2 - d)^2/2, 3/4 - d^2,
// (1/2 + d)^2/2. Order 3: start = floor(xi) - 1, weights (1-f)^3/6, (3f^3 - 6f^2 + 4)/6,
// (-3f^3 + 3f^2 + 3f + 1)/6, f^3/6.
template <int O>
__device__ __forceinline__ int nodal_weights(double xi, double* w) {
  if constexpr (O == 1) {
    const double i = floor(xi), f = xi - i;
    w[0] = 1.0 - f;
    w[1] = f;
    return (int)i;
  } else if constexpr (O == 2) {
    const double m = floor(xi + 0.5), d = xi - m;
    const double l = 0.5 - d, r = 0.5 + d;
    w[0] = 0.5 * (l * l);
    w[1] = 0.75 - d * d;
    w[2] = 0.5 * (r * r);
    return (int)m - 1;
  } else {
    const double i = floor(xi), f = xi - i, g = 1.0 - f;
    const double f2 = f * f, f3 = f2 * f;
    constexpr double s6 = 1.0 / 6.0;
    w[0] = s6 * (g * g * g);
    w[1] = s6 * (3.0 * f3 - 6.0 * f2 + 4.0);
    w[2] = s6 * (-3.0 * f3 + 3.0 * f2 + 3.0 * f + 1.0);
    w[3] = s6 * f3;
    return (int)i - 1;
  }
}

// The O+1 weights of a stencil starting at `start` on the (O+2)-node box starting at
// `first` (start - first is 0 or 1).
template <int O>
__device__ __forceinline__ void on_box(int start, int first, const double* w, double* box) {
  const bool shifted = start != first;
#pragma unroll
  for (int j = 0; j < O + 2; ++j) {
    const double lo = j <= O ? w[j] : 0.0;
    const double hi = j >= 1 ? w[j - 1] : 0.0;
    box[j] = shifted ? hi : lo;
  }
}

__device__ __forceinline__ int esk_store(const KGrid& G, int d, int m) {
  if (G.per[d]) {
    m %= G.n[d];
    return m < 0 ? m + G.n[d] : m;
  }
  m += G.g[d];
  return (m >= 0 && m < G.N[d]) ? m : -1;
}

// Window of one component in LDS: W nodes per dimension from w0, stored with row pitch py
// and plane pitch pz. The pitches are padded to py = 20 and pz = 4 (mod 32), so that the
// 64 box nodes one consumer instruction touches fall into distinct LDS banks (x
// component) or at most two to a bank (y, z).
struct EskWin {
  int w0[3], W[3], py, pz, size;
};

__host__ __device__ __forceinline__ int esk_pitch(int need, int residue) {
  return need + (((residue - need) % 32) + 32) % 32;
}

__host__ __device__ __forceinline__ size_t esk_win_size(const int* W) {
  const int py = esk_pitch(W[0], 20);
  const int pz = esk_pitch(py * W[1], 4);
  return (size_t)pz * W[2];
}

__device__ __forceinline__ EskWin esk_window(const TileBox& tb, int dim, int ml) {
  EskWin w;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const bool used = d < dim;
    w.w0[d] = used ? tb.c0[d] - ml : 0;
    w.W[d] = used ? tb.e[d] + 2 * ml : 1;
  }
  w.py = esk_pitch(w.W[0], 20);
  w.pz = esk_pitch(w.py * w.W[1], 4);
  w.size = w.pz * w.W[2];
  return w;
}

struct EskArgs {
  const double* xo[3];   // positions before the move, slot order
  double sc[3];          // dx_d / dt
};

// One slot's inputs, loaded ahead of their use.
struct EskRaw {
  double xo[3], xn[3];
  float w, uz, ux, uy;
  bool valid;
};

template <int DIM>
__device__ __forceinline__ void esk_fetch(const KPart& P, const EskArgs& X, int s, bool in,
                                          EskRaw& r) {
  r.valid = in && P.id[s] != PIC_INVALID_ID;
  if (!r.valid) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) r.xo[d] = d < DIM ? X.xo[d][s] : 0.0;
  r.xn[0] = P.x[s];
  r.xn[1] = P.y[s];
  r.xn[2] = DIM == 3 ? P.z[s] : 0.0;
  r.w = P.w[s];
  if constexpr (DIM == 2) {
    r.ux = P.ux[s];
    r.uy = P.uy[s];
    r.uz = P.uz[s];
  }
}

// Factor vectors of one particle into rec (float32) and the box's first node per
// dimension. Returns false (with an error bit) for a non-finite or out-of-domain position
// or a move of a cell or more.
template <int O, int DIM>
__device__ __forceinline__ bool esk_prep(const KGrid& G, const EskArgs& X, const EskRaw& raw,
                                         float* rec, int* first, uint32_t& bad) {
  const double qw = (double)G.q * (double)raw.w;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double a = (raw.xo[d] - G.x0[d]) * G.inv_dx[d];
    const double b0 = (raw.xn[d] - G.x0[d]) * G.inv_dx[d];
    if (!isfinite(a) || !isfinite(b0)) {
      bad |= PIC_EF_NONFINITE;
      return false;
    }
    const double n = (double)G.n[d];
    if (!(a >= 0.0 && a <= n && b0 >= 0.0 && b0 <= n)) {
      bad |= PIC_EF_DOMAIN;
      return false;
    }
    double step = b0 - a;
    if (G.per[d]) {            // nearest periodic image (|step| < n)
      if (step > 0.5 * n) step -= n;
      else if (step < -0.5 * n) step += n;
    }
    if (!(fabs(step) < 1.0)) {
      bad |= PIC_EF_MOVE;
      return false;
    }
    const double b = a + step;
    double w0[O + 1], w1[O + 1], s0[O + 2], s1[O + 2];
    const int st0 = nodal_weights<O>(a, w0);
    const int st1 = nodal_weights<O>(b, w1);
    const int f = min(st0, st1);
    first[d] = f;
    on_box<O>(st0, f, w0, s0);
    on_box<O>(st1, f, w1, s1);
    float* M = rec + 2 + d * (3 * O + 5);
    float* DS = M + (O + 2);
    float* A = DS + (O + 2);
    const double scale = -qw * X.sc[d];
    double run = 0.0;
#pragma unroll
    for (int k = 0; k < O + 2; ++k) {
      const double ds = s1[k] - s0[k];
      M[k] = (float)(0.5 * (s0[k] + s1[k]));
      DS[k] = (float)ds;
      if (k < O + 1) {
        run += ds;
        A[k] = (float)(scale * run);
      }
    }
  }
  if constexpr (DIM == 2) {
    const float ux = raw.ux, uy = raw.uy, uz = raw.uz;
    rec[1] = (float)qw * uz / sqrtf(1.0f + (ux * ux + uy * uy + uz * uz));
  } else {
    rec[1] = 0.0f;
  }
  return true;
}

// Value of box task (o0, o1, o2) of component C from a record.
template <int O, int DIM, int C>
__device__ __forceinline__ float esk_value(const float* rec, const int* o) {
  constexpr int RS = 3 * O + 5;
  const float* base = rec + 2;
  if constexpr (DIM == 3) {
    constexpr int D1 = (C + 1) % 3, D2 = (C + 2) % 3;
    const float a = base[C * RS + 2 * (O + 2) + o[C]];
    const float m1 = base[D1 * RS + o[D1]], m2 = base[D2 * RS + o[D2]];
    const float d1 = base[D1 * RS + (O + 2) + o[D1]], d2 = base[D2 * RS + (O + 2) + o[D2]];
    return a * (m1 * m2 + (1.0f / 12.0f) * (d1 * d2));
  } else if constexpr (C < 2) {
    constexpr int D1 = 1 - C;
    return base[C * RS + 2 * (O + 2) + o[C]] * base[D1 * RS + o[D1]];
  } else {
    const float mx = base[o[0]], my = base[RS + o[1]];
    const float dx = base[(O + 2) + o[0]], dy = base[RS + (O + 2) + o[1]];
    return rec[1] * (mx * my + (1.0f / 12.0f) * (dx * dy));
  }
}

// Component C of one particle's box added to J with global atomics. With REG (a record
// held in registers) the loops are unrolled so that every index is a compile-time
// constant; a record in LDS is read with plain loops.
template <int O, int DIM, int C, bool REG>
__device__ __forceinline__ void esk_global_comp(const KGrid& G, const float* rec,
                                                const int* first, float* J, uint32_t& bad) {
  constexpr int NX = esk_ext<O, DIM, C, 0>(), NY = esk_ext<O, DIM, C, 1>();
  constexpr int NT = NX * NY * esk_ext<O, DIM, C, 2>();
#pragma unroll (REG ? NT : 1)
  for (int t = 0; t < NT; ++t) {
    const int ox = t % NX, oy = (t / NX) % NY, oz = t / (NX * NY);
    const int o[3] = {ox, oy, oz};
    const float v = esk_value<O, DIM, C>(rec, o);
    const int ix = esk_store(G, 0, first[0] + ox);
    const int iy = esk_store(G, 1, first[1] + oy);
    const int iz = DIM == 3 ? esk_store(G, 2, first[2] + oz) : 0;
    if ((ix | iy | iz) < 0) {
      if (v != 0.0f) bad |= PIC_EF_STENCIL;
      continue;
    }
    unsafeAtomicAdd(&J[((int64_t)iz * G.N[1] + iy) * G.N[0] + ix], v);
  }
}

template <int O, int DIM, bool REG>
__device__ __forceinline__ void esk_global(const KGrid& G, const float* rec, const int* first,
                                           float* J0, float* J1, float* J2, uint32_t& bad) {
  esk_global_comp<O, DIM, 0, REG>(G, rec, first, J0, bad);
  esk_global_comp<O, DIM, 1, REG>(G, rec, first, J1, bad);
  esk_global_comp<O, DIM, 2, REG>(G, rec, first, J2, bad);
}

// One particle per lane, global atomics (no bins).
template <int O, int DIM>
__global__ __launch_bounds__(256) void k_esk_global(KGrid G, KPart P, EskArgs X, float* J0,
                                                    float* J1, float* J2, uint32_t* err) {
  uint32_t bad = 0;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < P.nslots; s += gridDim.x * blockDim.x) {
    EskRaw raw;
    esk_fetch<DIM>(P, X, s, true, raw);
    if (!raw.valid) continue;
    float rec[esk_rec<O, DIM>()];
    int first[3] = {0, 0, 0};
    if (esk_prep<O, DIM>(G, X, raw, rec, first, bad))
      esk_global<O, DIM, true>(G, rec, first, J0, J1, J2, bad);
  }
  if (bad) atomicOr(err, bad);
}

template <int O, int DIM>
struct EskLayout {
  size_t win_off, rec_off, lst_off, cnt_off, total;
  __host__ __device__ EskLayout(const int* T, int dim) {
    int Wm[3];
    for (int d = 0; d < 3; ++d) Wm[d] = d < dim ? T[d] + 2 * esk_margin<O>() : 1;
    const size_t ws = esk_win_size(Wm);
    win_off = 0;
    rec_off = 3 * ws * sizeof(float);
    lst_off = rec_off + 2 * (size_t)ESK_CHUNK * esk_rec<O, DIM>() * sizeof(float);
    cnt_off = lst_off + 2 * (size_t)ESK_CHUNK * sizeof(int);
    total = cnt_off + 2 * sizeof(int);
  }
};

// Wave C adds component C of the `n` listed records into its window.
template <int O, int DIM, int C>
__device__ __forceinline__ void esk_consume(const float* __restrict__ recs,
                                            const int* __restrict__ lst, int n,
                                            const EskWin& w, float* __restrict__ win) {
  constexpr int R = esk_rec<O, DIM>();
  constexpr int sz[3] = {esk_ext<O, DIM, C, 0>(), esk_ext<O, DIM, C, 1>(),
                         esk_ext<O, DIM, C, 2>()};
  constexpr int T = sz[0] * sz[1] * sz[2];
  const int lane = threadIdx.x % PIC_WAVE;
  float* wc = win + C * w.size;
  for (int pass = 0; pass * PIC_WAVE < T; ++pass) {
    const int t = lane + pass * PIC_WAVE;
    const bool act = t < T;
    const int o[3] = {t % sz[0], (t / sz[0]) % sz[1], t / (sz[0] * sz[1])};
    const int loff = o[2] * w.pz + o[1] * w.py + o[0];
#pragma unroll 4
    for (int p = 0; p < n; ++p) {
      const float* r = recs + lst[p] * R;
      if (act) {
        const int idx = __float_as_int(r[0]) + loff;
        wc[idx] += esk_value<O, DIM, C>(r, o);
      }
    }
  }
}

// Producer lane: the particle of slot S0 + 64 k + lane (already fetched into raw) prepared
// into the lane's record of buffer k & 1; records whose box fits the window are listed for
// the consumers, the others are added to J from here.
template <int O, int DIM>
__device__ __forceinline__ void esk_stage(const KGrid& G, const EskArgs& X, const EskRaw& raw,
                                          const EskWin& w, int k, float* recs, int* lst,
                                          int* cnt, float* J0, float* J1, float* J2,
                                          uint32_t& bad) {
  constexpr int R = esk_rec<O, DIM>();
  const int lane = threadIdx.x % PIC_WAVE;
  float* q = recs + ((k & 1) * ESK_CHUNK + lane) * R;
  float rec[R];
  int first[3] = {0, 0, 0};
  const bool ok = raw.valid && esk_prep<O, DIM>(G, X, raw, rec, first, bad);
  bool fits = ok;
  if (ok) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int r = first[d] - w.w0[d];
      fits = fits && r >= 0 && r + O + 1 < w.W[d];
    }
    const int rz = DIM == 3 ? first[2] - w.w0[2] : 0;
    rec[0] = __int_as_float(rz * w.pz + (first[1] - w.w0[1]) * w.py + (first[0] - w.w0[0]));
#pragma unroll
    for (int i = 0; i < R; ++i) q[i] = rec[i];
  }
  if (ok && !fits) esk_global<O, DIM, false>(G, q, first, J0, J1, J2, bad);
  const unsigned long long m = __ballot(fits);
  const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                             __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
  if (fits) lst[(k & 1) * ESK_CHUNK + rank] = lane;
  if (lane == 0) cnt[k & 1] = (int)__popcll(m);
}

template <int O, int DIM>
__global__ __launch_bounds__(ESK_WAVES* PIC_WAVE) void k_esk_tile(KGrid G, KBins B, KPart P,
                                                                  EskArgs X, float* J0,
                                                                  float* J1, float* J2) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int R = esk_rec<O, DIM>();
  constexpr int ML = esk_margin<O>();
  const EskLayout<O, DIM> L(B.T, DIM);
  float* win = (float*)(smem + L.win_off);
  float* recs = (float*)(smem + L.rec_off);
  int* lst = (int*)(smem + L.lst_off);
  int* cnt = (int*)(smem + L.cnt_off);
  const TileBox tb = tile_box(G.n, B.T, B.nt, blockIdx.x);
  const EskWin w = esk_window(tb, DIM, ML);
  const int wave = threadIdx.x / PIC_WAVE;
  const int lane = threadIdx.x % PIC_WAVE;
  for (int i = threadIdx.x; i < 3 * w.size; i += blockDim.x) win[i] = 0.0f;
  const int S0 = B.off[tb.b0], S1 = B.off[tb.b0 + tb.nb];
  const int nchunk = (S1 - S0 + ESK_CHUNK - 1) / ESK_CHUNK;
  uint32_t bad = 0;
  __syncthreads();
  if (wave == ESK_WAVES - 1) {
    // the next chunk's loads are in flight while the current one is prepared
    EskRaw cur, nxt;
    esk_fetch<DIM>(P, X, S0 + lane, S0 + lane < S1, cur);
    esk_fetch<DIM>(P, X, S0 + ESK_CHUNK + lane, S0 + ESK_CHUNK + lane < S1, nxt);
    if (nchunk > 0) esk_stage<O, DIM>(G, X, cur, w, 0, recs, lst, cnt, J0, J1, J2, bad);
    __syncthreads();
    for (int k = 0; k < nchunk; ++k) {
      if (k + 1 < nchunk) {
        cur = nxt;
        const int s2 = S0 + (k + 2) * ESK_CHUNK + lane;
        esk_fetch<DIM>(P, X, s2, s2 < S1, nxt);
        esk_stage<O, DIM>(G, X, cur, w, k + 1, recs, lst, cnt, J0, J1, J2, bad);
      }
      __syncthreads();
    }
  } else {
    __syncthreads();
    for (int k = 0; k < nchunk; ++k) {
      const float* rk = recs + (k & 1) * ESK_CHUNK * R;
      const int* lk = lst + (k & 1) * ESK_CHUNK;
      const int n = cnt[k & 1];
      if (wave == 0) esk_consume<O, DIM, 0>(rk, lk, n, w, win);
      else if (wave == 1) esk_consume<O, DIM, 1>(rk, lk, n, w, win);
      else esk_consume<O, DIM, 2>(rk, lk, n, w, win);
      __syncthreads();
    }
  }
  __syncthreads();
  // window -> J, one atomic per non-zero entry
  for (int i = threadIdx.x; i < 3 * w.size; i += blockDim.x) {
    const float v = win[i];
    if (v == 0.0f) continue;
    const int c = i / w.size;
    const int r = i - c * w.size;
    const int wz = r / w.pz, wy = (r - wz * w.pz) / w.py, wx = r - wz * w.pz - wy * w.py;
    if (wx >= w.W[0] || wy >= w.W[1]) continue;   // padding
    const int ix = esk_store(G, 0, w.w0[0] + wx), iy = esk_store(G, 1, w.w0[1] + wy);
    const int iz = DIM == 3 ? esk_store(G, 2, w.w0[2] + wz) : 0;
    if ((ix | iy | iz) < 0) {
      bad |= PIC_EF_STENCIL;
      continue;
    }
    float* Jc = c == 0 ? J0 : (c == 1 ? J1 : J2);
    unsafeAtomicAdd(&Jc[((int64_t)iz * G.N[1] + iy) * G.N[0] + ix], v);
  }
  if (bad) atomicOr(B.err, bad);
}

template <int O, int DIM>
void launch_esk(const KGrid& G, const KPart& P, pic_bins* b, const EskArgs& X, float* J0,
                float* J1, float* J2, hipStream_t s) {
  if (b && b->sorted_once) {
    const EskLayout<O, DIM> L(b->kb.T, DIM);
    if (L.total <= b->max_lds) {
      hipLaunchKernelGGL((k_esk_tile<O, DIM>), dim3(b->kb.ntiles), dim3(ESK_WAVES * PIC_WAVE),
                         L.total, s, G, b->kb, P, X, J0, J1, J2);
      return;
    }
  }
  const unsigned blocks = (unsigned)std::min<int64_t>(((int64_t)P.nslots + 255) / 256, 16384);
  if (blocks == 0) return;
  hipLaunchKernelGGL((k_esk_global<O, DIM>), dim3(blocks), dim3(256), 0, s, G, P, X, J0, J1, J2,
                     b ? b->kb.err : nobins_err_ptr());
}

}  // namespace

extern "C" pic_status pic_deposit_esirkepov(const pic_grid* grid, const pic_particles* p,
                                            pic_bins* b, const double* x_old,
                                            const double* y_old, const double* z_old,
                                            float* Jx, float* Jy, float* Jz, unsigned flags,
                                            hipStream_t stream) {
  pic_status st = validate_grid(grid);
  if (st != PIC_OK) return st;
  if ((st = validate_particles(p, grid->dim)) != PIC_OK) return st;
  if (!Jx || !Jy || !Jz) return set_error(PIC_ERR_INVALID_ARG, "J pointers must not be NULL");
  if (p->nslots > 0 && (!x_old || !y_old || (grid->dim == 3 && !z_old)))
    return set_error(PIC_ERR_INVALID_ARG, "old position pointers must not be NULL");
  if (flags & ~(unsigned)PIC_F_ACCUMULATE)
    return set_error(PIC_ERR_INVALID_ARG, "pic_deposit_esirkepov takes PIC_F_ACCUMULATE only");
  if (!std::isfinite(grid->dt) || grid->dt == 0.0)
    return set_error(PIC_ERR_INVALID_ARG, "dt must be finite and non-zero");
  if (b) {
    if (!same_grid(*grid, b->grid)) return set_error(PIC_ERR_INVALID_ARG, "grid differs from the bins' grid");
    if (p->nslots != b->nslots) return set_error(PIC_ERR_INVALID_ARG, "nslots differs from the bins' nslots");
  }
  const KGrid G = make_kgrid(*grid);
  const KPart P = make_kpart(*p);
  EskArgs X{{x_old, y_old, grid->dim == 3 ? z_old : x_old}, {0.0, 0.0, 0.0}};
  for (int d = 0; d < grid->dim; ++d) X.sc[d] = grid->dx[d] / grid->dt;
  const int64_t nJ = (int64_t)G.N[0] * G.N[1] * G.N[2];
  if (!(flags & PIC_F_ACCUMULATE)) {
    launch_zero_j3(Jx, Jy, Jz, nJ, stream);
  }
#define ES(O_, D_) launch_esk<O_, D_>(G, P, b, X, Jx, Jy, Jz, stream)
  if (G.dim == 3) {
    if (G.order == 1) ES(1, 3); else if (G.order == 2) ES(2, 3); else ES(3, 3);
  } else {
    if (G.order == 1) ES(1, 2); else if (G.order == 2) ES(2, 2); else ES(3, 2);
  }
#undef ES
  return check_hip(hipGetLastError(), "pic_deposit_esirkepov launch");
}
