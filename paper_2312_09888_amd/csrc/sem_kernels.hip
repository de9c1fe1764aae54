// HIP kernels of the extraction path (gfx950), generic over the order N.
//
// Per element (Deville, Fischer & Mund 2002, ch. 4; Hunt, Wray & Moin 1988):
//   reference derivatives  f_r = D f (along i), f_s (along j), f_t (along k)
//   Jacobian               J = d(x,y,z)/d(r,s,t), J^-1 = adj(J) / det J
//   chain rule             A_ij = sum_a (d u_i / d r_a) (J^-1)_{a j}
//   Q = -tr(A^2)/2 (equal to Hunt's (|Omega|^2 - |S|^2)/2), |omega|.
// Marching cubes over the N^3 sub-hexahedra (Lorensen & Cline 1987) with a
// count / exclusive-scan / emit compaction.
//
// Every 1-D contraction subtracts the line's first value before applying D:
// sum_m D_im (f_m - f_0) equals (D f)_i exactly in exact arithmetic because
// D annihilates constants, but it removes the large common offset of
// coordinates and velocities before rounding.  In FP32 this is what keeps
// the Jacobian of a small element at a large absolute position accurate.
#include <cmath>
#include <cstdint>

#include "sem_internal.h"

namespace sem {
namespace {

template <int N>
struct Shape {
  static constexpr int P = N + 1;
  static constexpr int NP = P * P * P;                // nodes per element
  static constexpr int NC = N * N * N;                // cells per element
  static constexpr int kNodeThreads = ((NP + 63) / 64) * 64;
  static constexpr int kCellThreads = ((NC + 63) / 64) * 64;
};

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T neg_inf() { return -__builtin_huge_val(); }
template <>
__device__ __forceinline__ float neg_inf<float>() { return -__builtin_huge_valf(); }
template <typename T>
__device__ __forceinline__ T pos_inf() { return -neg_inf<T>(); }

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off);
    v = o < v ? o : v;
  }
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Block-wide (min, max) of per-thread values; result valid in every thread.
template <typename T, int THREADS>
__device__ __forceinline__ void block_minmax(T& mn, T& mx, T* scratch /*2*THREADS/64*/) {
  constexpr int W = THREADS / 64;
  mn = wave_min(mn);
  mx = wave_max(mx);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    scratch[w] = mn;
    scratch[W + w] = mx;
  }
  __syncthreads();
  mn = scratch[0];
  mx = scratch[W];
#pragma unroll
  for (int i = 1; i < W; ++i) {
    mn = scratch[i] < mn ? scratch[i] : mn;
    mx = scratch[W + i] > mx ? scratch[W + i] : mx;
  }
  __syncthreads();
}

// Block-wide sum of a 64-bit value; result valid in every thread.
template <int THREADS>
__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t* scratch /*THREADS/64*/) {
  constexpr int W = THREADS / 64;
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
  __syncthreads();
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < W; ++i) s += scratch[i];
  __syncthreads();
  return s;
}

// Exclusive block scan of a 64-bit value (THREADS multiple of 64).
template <int THREADS>
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t* scratch,
                                                        int64_t* total) {
  constexpr int W = THREADS / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int64_t o = __shfl_up(inc, off);
    if (lane >= off) inc += o;
  }
  if (lane == 63) scratch[w] = inc;
  __syncthreads();
  int64_t before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    before += (i < w) ? scratch[i] : 0;
    all += scratch[i];
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

// 1-D contractions at node (i, j, k) of a tile in LDS, line-shifted.
template <int N, typename T>
__device__ __forceinline__ void ref_derivs(const T* __restrict__ f, const T* __restrict__ d,
                                           int i, int j, int k, T& fr, T& fs, T& ft) {
  constexpr int P = N + 1;
  const T* lr = f + (k * P + j) * P;   // line along i
  const T* ls = f + k * P * P + i;     // along j, stride P
  const T* lt = f + j * P + i;         // along k, stride P^2
  const T r0 = lr[0], s0 = ls[0], t0 = lt[0];
  T ar = T(0), as = T(0), at = T(0);
#pragma unroll
  for (int m = 1; m < P; ++m) {
    ar = fma(d[i * P + m], lr[m] - r0, ar);
    as = fma(d[j * P + m], ls[m * P] - s0, as);
    at = fma(d[k * P + m], lt[m * P * P] - t0, at);
  }
  fr = ar;
  fs = as;
  ft = at;
}

template <typename T>
struct InvJac {
  T rx, ry, rz, sx, sy, sz, tx, ty, tz;
};

// J^-1 = adj(J) / det J; returns det J > 0.
template <typename T>
__device__ __forceinline__ bool invert_jacobian(T xr, T xs, T xt, T yr, T ys, T yt, T zr,
                                                T zs, T zt, InvJac<T>& k) {
  const T c0 = ys * zt - yt * zs;
  const T c1 = yt * zr - yr * zt;
  const T c2 = yr * zs - ys * zr;
  const T det = xr * c0 + xs * c1 + xt * c2;
  const T inv = T(1) / det;
  k.rx = c0 * inv;
  k.ry = (xt * zs - xs * zt) * inv;
  k.rz = (xs * yt - xt * ys) * inv;
  k.sx = c1 * inv;
  k.sy = (xr * zt - xt * zr) * inv;
  k.sz = (xt * yr - xr * yt) * inv;
  k.tx = c2 * inv;
  k.ty = (xs * zr - xr * zs) * inv;
  k.tz = (xr * ys - xs * yr) * inv;
  return det > T(0);
}

// ---------------------------------------------------------------------------
// gradient / Q-criterion: one workgroup per element, tiles staged in LDS
// ---------------------------------------------------------------------------

template <int N, typename T>
__global__ void __launch_bounds__(Shape<N>::kNodeThreads)
derivs_tile(const T* __restrict__ dmat, const T* __restrict__ x, const T* __restrict__ y,
            const T* __restrict__ z, const T* __restrict__ f, T* __restrict__ gx,
            T* __restrict__ gy, T* __restrict__ gz, int32_t* __restrict__ status) {
  using S = Shape<N>;
  __shared__ T sd[S::P * S::P];
  __shared__ T sf[4][S::NP];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * S::NP;
  if (t < S::P * S::P) sd[t] = dmat[t];
  if (t < S::NP) {
    sf[0][t] = x[base + t];
    sf[1][t] = y[base + t];
    sf[2][t] = z[base + t];
    sf[3][t] = f[base + t];
  }
  __syncthreads();
  int bad = 0;
  if (t < S::NP) {
    const int i = t % S::P, j = (t / S::P) % S::P, k = t / (S::P * S::P);
    T xr, xs, xt, yr, ys, yt, zr, zs, zt, fr, fs, ft;
    ref_derivs<N>(sf[0], sd, i, j, k, xr, xs, xt);
    ref_derivs<N>(sf[1], sd, i, j, k, yr, ys, yt);
    ref_derivs<N>(sf[2], sd, i, j, k, zr, zs, zt);
    ref_derivs<N>(sf[3], sd, i, j, k, fr, fs, ft);
    InvJac<T> kk;
    bad = !invert_jacobian(xr, xs, xt, yr, ys, yt, zr, zs, zt, kk);
    gx[base + t] = fr * kk.rx + fs * kk.sx + ft * kk.tx;
    gy[base + t] = fr * kk.ry + fs * kk.sy + ft * kk.ty;
    gz[base + t] = fr * kk.rz + fs * kk.sz + ft * kk.tz;
  }
  bad = __syncthreads_or(bad);
  if (bad && t == 0 && status) atomicOr(status, SEM_FLAG_BAD_JACOBIAN);
}

template <int N, typename T>
__global__ void __launch_bounds__(Shape<N>::kNodeThreads)
qcrit_tile(const T* __restrict__ dmat, const T* __restrict__ x, const T* __restrict__ y,
           const T* __restrict__ z, const T* __restrict__ u, const T* __restrict__ v,
           const T* __restrict__ w, T* __restrict__ q, T* __restrict__ om,
           T* __restrict__ qmm, int32_t* __restrict__ status) {
  using S = Shape<N>;
  __shared__ T sd[S::P * S::P];
  __shared__ T sf[6][S::NP];
  __shared__ T red[2 * (S::kNodeThreads / 64)];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * S::NP;
  if (t < S::P * S::P) sd[t] = dmat[t];
  if (t < S::NP) {
    sf[0][t] = x[base + t];
    sf[1][t] = y[base + t];
    sf[2][t] = z[base + t];
    sf[3][t] = u[base + t];
    sf[4][t] = v[base + t];
    sf[5][t] = w[base + t];
  }
  __syncthreads();
  int bad = 0;
  T qv = neg_inf<T>();
  if (t < S::NP) {
    const int i = t % S::P, j = (t / S::P) % S::P, k = t / (S::P * S::P);
    T xr, xs, xt, yr, ys, yt, zr, zs, zt;
    ref_derivs<N>(sf[0], sd, i, j, k, xr, xs, xt);
    ref_derivs<N>(sf[1], sd, i, j, k, yr, ys, yt);
    ref_derivs<N>(sf[2], sd, i, j, k, zr, zs, zt);
    InvJac<T> kk;
    bad = !invert_jacobian(xr, xs, xt, yr, ys, yt, zr, zs, zt, kk);
    T a[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T fr, fs, ft;
      ref_derivs<N>(sf[3 + c], sd, i, j, k, fr, fs, ft);
      a[c][0] = fr * kk.rx + fs * kk.sx + ft * kk.tx;
      a[c][1] = fr * kk.ry + fs * kk.sy + ft * kk.ty;
      a[c][2] = fr * kk.rz + fs * kk.sz + ft * kk.tz;
    }
    const T tr2 = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2] +
                  T(2) * (a[0][1] * a[1][0] + a[0][2] * a[2][0] + a[1][2] * a[2][1]);
    const T w1 = a[2][1] - a[1][2], w2 = a[0][2] - a[2][0], w3 = a[1][0] - a[0][1];
    qv = T(-0.5) * tr2;
    if (q) q[base + t] = qv;
    if (om) om[base + t] = sqrt(w1 * w1 + w2 * w2 + w3 * w3);
    if (qv != qv) qv = neg_inf<T>();
  }
  bad = __syncthreads_or(bad);
  if (bad && t == 0 && status) atomicOr(status, SEM_FLAG_BAD_JACOBIAN);
  if (qmm) {
    T mn = t < S::NP ? qv : pos_inf<T>();
    T mx = qv;
    block_minmax<T, S::kNodeThreads>(mn, mx, red);
    if (t == 0) {
      qmm[2 * (int64_t)blockIdx.x] = mn;
      qmm[2 * (int64_t)blockIdx.x + 1] = mx;
    }
  }
}

// ---------------------------------------------------------------------------
// marching cubes
// ---------------------------------------------------------------------------

// low corner and axis of each cube edge (edge id = 4*axis + rank)
__constant__ int8_t kEdgeLo[12] = {0, 2, 4, 6, 0, 1, 4, 5, 0, 1, 2, 3};
__constant__ int8_t kEdgeAxis[12] = {0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2, 2};

template <int P>
__device__ __forceinline__ int corner_offset(int v) {
  return (v & 1) + P * ((v >> 1) & 1) + P * P * ((v >> 2) & 1);
}

template <int N, typename T>
__device__ __forceinline__ int cell_case(const T* __restrict__ sf, int n0, T c) {
  constexpr int P = N + 1;
  int cs = 0;
#pragma unroll
  for (int vtx = 0; vtx < 8; ++vtx) cs |= (sf[n0 + corner_offset<P>(vtx)] > c) << vtx;
  return cs;
}

// Per (isovalue, element): triangle and active-cell counts; optional case dump.
template <int N, typename T>
__global__ void __launch_bounds__(Shape<N>::kCellThreads)
iso_count(int64_t n_elem, const T* __restrict__ field, const T* __restrict__ mm, int n_iso,
          IsoList<T> iso, const uint8_t* __restrict__ ntri_tab, int32_t* __restrict__ cnt,
          int64_t* __restrict__ active_total, uint8_t* __restrict__ case_idx) {
  using S = Shape<N>;
  constexpr int TH = S::kCellThreads;
  __shared__ T sf[S::NP];
  __shared__ uint8_t s_ntri[256];
  __shared__ T red[2 * (TH / 64)];
  __shared__ int64_t sred[TH / 64];
  const int t = threadIdx.x;
  const int64_t e = blockIdx.x;
  const int64_t base = e * S::NP;
  for (int q = t; q < 256; q += TH) s_ntri[q] = ntri_tab[q];
  T mn, mx;
  bool need = true;
  if (mm) {
    mn = mm[2 * e];
    mx = mm[2 * e + 1];
    need = false;
    for (int s = 0; s < n_iso; ++s) need = need || ((mx > iso.v[s]) && !(mn > iso.v[s]));
  }
  if (need)
    for (int q = t; q < S::NP; q += TH) sf[q] = field[base + q];
  __syncthreads();
  if (!mm) {
    T a = pos_inf<T>(), b = neg_inf<T>();
    for (int q = t; q < S::NP; q += TH) {
      T val = sf[q];
      if (val != val) val = neg_inf<T>();
      a = val < a ? val : a;
      b = val > b ? val : b;
    }
    block_minmax<T, TH>(a, b, red);
    mn = a;
    mx = b;
  }
  const int i = t % N, j = (t / N) % N, k = t / (N * N);
  const int n0 = i + S::P * (j + S::P * k);
  for (int s = 0; s < n_iso; ++s) {
    const T c = iso.v[s];
    const bool straddle = (mx > c) && !(mn > c);
    uint8_t* cdump = case_idx ? case_idx + ((int64_t)s * n_elem + e) * S::NC : nullptr;
    if (!straddle) {
      if (t == 0) cnt[(int64_t)s * n_elem + e] = 0;
      if (cdump && t < S::NC) cdump[t] = (mx > c) ? 255 : 0;
      continue;
    }
    int64_t nt = 0, act = 0;
    if (t < S::NC) {
      const int cs = cell_case<N>(sf, n0, c);
      nt = s_ntri[cs];
      act = (cs != 0 && cs != 255);
      if (cdump) cdump[t] = (uint8_t)cs;
    }
    nt = block_sum<TH>(nt, sred);
    act = block_sum<TH>(act, sred);
    if (t == 0) {
      cnt[(int64_t)s * n_elem + e] = (int32_t)nt;
      if (active_total && act) atomicAdd((unsigned long long*)&active_total[s],
                                         (unsigned long long)act);
    }
  }
}

// Emit triangles of every (isovalue, element) with a nonzero count.
template <int N, typename T>
__global__ void __launch_bounds__(Shape<N>::kCellThreads)
iso_emit(int64_t n_elem, const T* __restrict__ x, const T* __restrict__ y,
         const T* __restrict__ z, const T* __restrict__ field, int n_iso, IsoList<T> iso,
         const uint8_t* __restrict__ ntri_tab, const int8_t* __restrict__ tri_tab,
         const int32_t* __restrict__ cnt, const int64_t* __restrict__ offs,
         T* __restrict__ tri_xyz, int64_t cap, uint64_t* __restrict__ keys) {
  using S = Shape<N>;
  constexpr int TH = S::kCellThreads;
  constexpr int W = TH / 64;
  __shared__ T sf[S::NP], sx[S::NP], sy[S::NP], sz[S::NP];
  __shared__ uint8_t s_ntri[256];
  __shared__ int8_t s_tri[256 * kMcMaxTri * 3];
  __shared__ int32_t s_wave[W];
  const int t = threadIdx.x;
  const int64_t e = blockIdx.x;
  bool any = false;
  for (int s = 0; s < n_iso; ++s) any = any || cnt[(int64_t)s * n_elem + e] > 0;
  if (!any) return;
  const int64_t base = e * S::NP;
  for (int q = t; q < 256; q += TH) s_ntri[q] = ntri_tab[q];
  for (int q = t; q < 256 * kMcMaxTri * 3; q += TH) s_tri[q] = tri_tab[q];
  for (int q = t; q < S::NP; q += TH) {
    sf[q] = field[base + q];
    sx[q] = x[base + q];
    sy[q] = y[base + q];
    sz[q] = z[base + q];
  }
  __syncthreads();
  const int i = t % N, j = (t / N) % N, k = t / (N * N);
  const int n0 = i + S::P * (j + S::P * k);
  const int lane = t & 63, wv = t >> 6;
  for (int s = 0; s < n_iso; ++s) {
    const int64_t flat = (int64_t)s * n_elem + e;
    if (cnt[flat] == 0) continue;
    const T c = iso.v[s];
    int cs = 0, nt = 0;
    if (t < S::NC) {
      cs = cell_case<N>(sf, n0, c);
      nt = s_ntri[cs];
    }
    // wave prefix of the 3-bit counts from one ballot per bit
    const uint64_t m0 = __ballot(nt & 1), m1 = __ballot(nt & 2), m2 = __ballot(nt & 4);
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int pre = __popcll(m0 & lt) + 2 * __popcll(m1 & lt) + 4 * __popcll(m2 & lt);
    if (lane == 0) s_wave[wv] = __popcll(m0) + 2 * __popcll(m1) + 4 * __popcll(m2);
    __syncthreads();
    int64_t g = offs[flat] + pre;
    for (int q = 0; q < wv; ++q) g += s_wave[q];
    for (int slot = 0; slot < nt; ++slot, ++g) {
      if (g >= cap) break;
      T* out = tri_xyz + g * 9;
#pragma unroll
      for (int vtx = 0; vtx < 3; ++vtx) {
        const int edge = s_tri[(cs * kMcMaxTri + slot) * 3 + vtx];
        const int lo = n0 + corner_offset<S::P>(kEdgeLo[edge]);
        const int ax = kEdgeAxis[edge];
        const int hi = lo + (ax == 0 ? 1 : ax == 1 ? S::P : S::P * S::P);
        {
#pragma clang fp contract(off)
          const T f0 = sf[lo], f1 = sf[hi];
          const T tt = (c - f0) / (f1 - f0);
          out[3 * vtx + 0] = sx[lo] + tt * (sx[hi] - sx[lo]);
          out[3 * vtx + 1] = sy[lo] + tt * (sy[hi] - sy[lo]);
          out[3 * vtx + 2] = sz[lo] + tt * (sz[hi] - sz[lo]);
        }
        if (keys) keys[g * 3 + vtx] = ((uint64_t)(base + lo)) * 3u + (uint64_t)ax;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan of int32 counts into int64 offsets
// ---------------------------------------------------------------------------

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ void __launch_bounds__(kScanThreads)
scan_reduce(const int32_t* __restrict__ cnt, int64_t count, int64_t* __restrict__ partial) {
  __shared__ int64_t sred[kScanThreads / 64];
  const int64_t start = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const int64_t idx = start + r * kScanThreads + threadIdx.x;
    if (idx < count) s += cnt[idx];
  }
  s = block_sum<kScanThreads>(s, sred);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(1024)
scan_partials(int64_t* __restrict__ partial, int64_t nb) {
  __shared__ int64_t sred[1024 / 64];
  int64_t running = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
    const int64_t idx = c0 + threadIdx.x;
    const int64_t v = idx < nb ? partial[idx] : 0;
    int64_t total;
    const int64_t ex = block_exclusive_scan<1024>(v, sred, &total);
    if (idx < nb) partial[idx] = running + ex;
    running += total;
  }
  if (threadIdx.x == 0) partial[nb] = running;
}

__global__ void __launch_bounds__(kScanThreads)
scan_apply(const int32_t* __restrict__ cnt, int64_t count, const int64_t* __restrict__ partial,
           int64_t nb, int64_t* __restrict__ offs) {
  __shared__ int64_t sred[kScanThreads / 64];
  const int64_t start = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    v[r] = (start + r < count) ? cnt[start + r] : 0;
    s += v[r];
  }
  int64_t total;
  int64_t run = partial[blockIdx.x] + block_exclusive_scan<kScanThreads>(s, sred, &total);
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    if (start + r < count) offs[start + r] = run;
    run += v[r];
  }
  if (blockIdx.x == nb - 1 && threadIdx.x == 0) offs[count] = partial[nb];
}

__global__ void iso_totals(const int64_t* __restrict__ offs, int64_t n_elem, int n_iso,
                           int64_t* __restrict__ tri_count, int64_t cap,
                           int32_t* __restrict__ status) {
  const int s = threadIdx.x;
  if (s < n_iso) tri_count[s] = offs[(int64_t)(s + 1) * n_elem] - offs[(int64_t)s * n_elem];
  if (s == 0 && status && offs[(int64_t)n_iso * n_elem] > cap)
    atomicOr(status, SEM_FLAG_TRI_OVERFLOW);
}

__global__ void fill_i64(int64_t* __restrict__ p, int n, int64_t value) {
  const int s = threadIdx.x;
  if (s < n) p[s] = value;
}

// ---------------------------------------------------------------------------
// dispatch over the order
// ---------------------------------------------------------------------------

#define SEM_ORDER_SWITCH(order, BODY) \
  switch (order) {                    \
    case 1: { constexpr int N = 1; BODY; } break; \
    case 2: { constexpr int N = 2; BODY; } break; \
    case 3: { constexpr int N = 3; BODY; } break; \
    case 4: { constexpr int N = 4; BODY; } break; \
    case 5: { constexpr int N = 5; BODY; } break; \
    case 6: { constexpr int N = 6; BODY; } break; \
    case 7: { constexpr int N = 7; BODY; } break; \
    case 8: { constexpr int N = 8; BODY; } break; \
    case 9: { constexpr int N = 9; BODY; } break; \
    default: return hipErrorInvalidValue;          \
  }

template <typename T>
const T* dmat_of(const DeviceTables& tab, int order);
template <>
const double* dmat_of<double>(const DeviceTables& tab, int order) { return tab.d64[order]; }
template <>
const float* dmat_of<float>(const DeviceTables& tab, int order) { return tab.d32[order]; }

template <typename T>
hipError_t derivs_t(int order, const DeviceTables& tab, int64_t n_elem, const void* x,
                    const void* y, const void* z, const void* f, void* gx, void* gy, void* gz,
                    int32_t* status, hipStream_t s) {
  const T* d = dmat_of<T>(tab, order);
  SEM_ORDER_SWITCH(order, {
    hipLaunchKernelGGL((derivs_tile<N, T>), dim3((unsigned)n_elem),
                       dim3(Shape<N>::kNodeThreads), 0, s, d, (const T*)x, (const T*)y,
                       (const T*)z, (const T*)f, (T*)gx, (T*)gy, (T*)gz, status);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t qcrit_t(int order, const DeviceTables& tab, int64_t n_elem, const void* x,
                   const void* y, const void* z, const void* u, const void* v, const void* w,
                   void* q, void* om, void* qmm, int32_t* status, hipStream_t s) {
  const T* d = dmat_of<T>(tab, order);
  SEM_ORDER_SWITCH(order, {
    hipLaunchKernelGGL((qcrit_tile<N, T>), dim3((unsigned)n_elem),
                       dim3(Shape<N>::kNodeThreads), 0, s, d, (const T*)x, (const T*)y,
                       (const T*)z, (const T*)u, (const T*)v, (const T*)w, (T*)q, (T*)om,
                       (T*)qmm, status);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t iso_t(int order, const DeviceTables& tab, int64_t n_elem, const void* x,
                 const void* y, const void* z, const void* field, const void* mm, int n_iso,
                 const double* iso_host, void* tri_xyz, int64_t cap, uint64_t* keys,
                 int64_t* tri_count, int64_t* active, uint8_t* case_idx,
                 const IsoWorkspace& ws, int32_t* status, hipStream_t s) {
  IsoList<T> iso;
  for (int q = 0; q < SEM_MAX_ISO; ++q) iso.v[q] = q < n_iso ? (T)iso_host[q] : T(0);
  if (active) hipLaunchKernelGGL(fill_i64, dim3(1), dim3(64), 0, s, active, n_iso, (int64_t)0);
  const int64_t count = (int64_t)n_iso * n_elem;
  const int64_t nb = scan_blocks(count);
  SEM_ORDER_SWITCH(order, {
    hipLaunchKernelGGL((iso_count<N, T>), dim3((unsigned)n_elem),
                       dim3(Shape<N>::kCellThreads), 0, s, n_elem, (const T*)field,
                       (const T*)mm, n_iso, iso, tab.ntri, ws.cnt, active, case_idx);
  });
  hipLaunchKernelGGL(scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, ws.cnt, count,
                     ws.partial);
  hipLaunchKernelGGL(scan_partials, dim3(1), dim3(1024), 0, s, ws.partial, nb);
  hipLaunchKernelGGL(scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s, ws.cnt, count,
                     ws.partial, nb, ws.offs);
  hipLaunchKernelGGL(iso_totals, dim3(1), dim3(SEM_MAX_ISO), 0, s, ws.offs, n_elem, n_iso,
                     tri_count, cap, status);
  if (cap > 0) {
    SEM_ORDER_SWITCH(order, {
      hipLaunchKernelGGL((iso_emit<N, T>), dim3((unsigned)n_elem),
                         dim3(Shape<N>::kCellThreads), 0, s, n_elem, (const T*)x,
                         (const T*)y, (const T*)z, (const T*)field, n_iso, iso, tab.ntri,
                         tab.tri, ws.cnt, ws.offs, (T*)tri_xyz, cap, keys);
    });
  }
  return hipGetLastError();
}

}  // namespace

int64_t scan_blocks(int64_t count) { return count <= 0 ? 1 : (count + kScanTile - 1) / kScanTile; }

hipError_t launch_derivs(int order, sem_dtype dt, const DeviceTables& tab, int64_t n_elem,
                         const void* x, const void* y, const void* z, const void* f, void* gx,
                         void* gy, void* gz, int32_t* status, hipStream_t s) {
  return dt == SEM_F64 ? derivs_t<double>(order, tab, n_elem, x, y, z, f, gx, gy, gz, status, s)
                       : derivs_t<float>(order, tab, n_elem, x, y, z, f, gx, gy, gz, status, s);
}

hipError_t launch_qcrit(int order, sem_dtype dt, const DeviceTables& tab, int64_t n_elem,
                        const void* x, const void* y, const void* z, const void* u,
                        const void* v, const void* w, void* q, void* om, void* qmm,
                        int32_t* status, hipStream_t s) {
  return dt == SEM_F64
             ? qcrit_t<double>(order, tab, n_elem, x, y, z, u, v, w, q, om, qmm, status, s)
             : qcrit_t<float>(order, tab, n_elem, x, y, z, u, v, w, q, om, qmm, status, s);
}

hipError_t launch_isosurface(int order, sem_dtype dt, const DeviceTables& tab, int64_t n_elem,
                             const void* x, const void* y, const void* z, const void* field,
                             const void* mm, int n_iso, const double* iso_host, void* tri_xyz,
                             int64_t cap, uint64_t* keys, int64_t* tri_count,
                             int64_t* active, uint8_t* case_idx, const IsoWorkspace& ws,
                             int32_t* status, hipStream_t s) {
  if (n_elem == 0) {
    hipLaunchKernelGGL(fill_i64, dim3(1), dim3(64), 0, s, tri_count, n_iso, (int64_t)0);
    if (active) hipLaunchKernelGGL(fill_i64, dim3(1), dim3(64), 0, s, active, n_iso, (int64_t)0);
    return hipGetLastError();
  }
  return dt == SEM_F64
             ? iso_t<double>(order, tab, n_elem, x, y, z, field, mm, n_iso, iso_host, tri_xyz,
                             cap, keys, tri_count, active, case_idx, ws, status, s)
             : iso_t<float>(order, tab, n_elem, x, y, z, field, mm, n_iso, iso_host, tri_xyz,
                            cap, keys, tri_count, active, case_idx, ws, status, s);
}

}  // namespace sem
