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
#include <mutex>
#include <unordered_map>
#include <type_traits>

#include <hip/hip_ext.h>

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

// One DPP move of a 32- or 64-bit value (a 64-bit value as its two halves
// under the same control).  With every row enabled each lane reads a lane of
// its own row; lanes of rows that ROWS leaves out keep `fill`.
template <int CTRL, typename T>
__device__ __forceinline__ T dpp_move(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(
        T, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xf, 0xf, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}
template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ T dpp_move(T v, T fill) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, fill),
                                                             __builtin_bit_cast(int, v), CTRL,
                                                             ROWS, 0xf, false));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, v), f = __builtin_bit_cast(uint64_t, fill);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(
        (int)(uint32_t)f, (int)(uint32_t)u, CTRL, ROWS, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(
        (int)(uint32_t)(f >> 32), (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xf, false);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}

// Minimum and maximum over the wave, left in lane 63 (other lanes hold
// partial results), by DPP moves only: within quads (quad_perm [1,0,3,2],
// [2,3,0,1]), half rows (row_half_mirror), rows (row_mirror), then lane 15
// of rows 0 and 2 into rows 1 and 3 (row_bcast:15) and lane 31 into rows 2
// and 3 (row_bcast:31).  No NaN may reach it: callers map NaN to -inf.
template <typename T>
__device__ __forceinline__ void wave_minmax(T& mn, T& mx) {
  const T pinf = pos_inf<T>(), ninf = neg_inf<T>();
  mn = fmin(mn, dpp_move<0xb1>(mn));
  mx = fmax(mx, dpp_move<0xb1>(mx));
  mn = fmin(mn, dpp_move<0x4e>(mn));
  mx = fmax(mx, dpp_move<0x4e>(mx));
  mn = fmin(mn, dpp_move<0x141>(mn));
  mx = fmax(mx, dpp_move<0x141>(mx));
  mn = fmin(mn, dpp_move<0x140>(mn));
  mx = fmax(mx, dpp_move<0x140>(mx));
  mn = fmin(mn, dpp_move<0x142, 0xa>(mn, pinf));
  mx = fmax(mx, dpp_move<0x142, 0xa>(mx, ninf));
  mn = fmin(mn, dpp_move<0x143, 0xc>(mn, pinf));
  mx = fmax(mx, dpp_move<0x143, 0xc>(mx, ninf));
}
// Inclusive sum of a 64-bit value over the lanes up to this one (lane 63:
// the wave's sum), by DPP moves of both halves: row shifts right by 1, 2,
// 4, 8 (lanes without a source add 0), then lane 15 of rows 0 and 2 into
// rows 1 and 3 (row_bcast:15) and lane 31 into rows 2 and 3
// (row_bcast:31).  Every lane of the wave must be active.
__device__ __forceinline__ int64_t wave_inclusive_sum(int64_t v) {
  const int64_t z = 0;
  v += dpp_move<0x111, 0xf>(v, z);
  v += dpp_move<0x112, 0xf>(v, z);
  v += dpp_move<0x114, 0xf>(v, z);
  v += dpp_move<0x118, 0xf>(v, z);
  v += dpp_move<0x142, 0xa>(v, z);
  v += dpp_move<0x143, 0xc>(v, z);
  return v;
}

// Block-wide (min, max) of per-thread values; result valid in every thread.
template <typename T, int THREADS>
__device__ __forceinline__ void block_minmax(T& mn, T& mx, T* scratch /*2*THREADS/64*/) {
  constexpr int W = THREADS / 64;
  wave_minmax(mn, mx);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) {
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
  v = wave_inclusive_sum(v);
  if ((threadIdx.x & 63) == 63) scratch[threadIdx.x >> 6] = v;
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
  const int64_t inc = wave_inclusive_sum(v);
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

// A value the compiler can no longer trace to its source (no instruction).
template <typename V>
__device__ __forceinline__ V opaque(V x) {
  asm("" : "+v"(x));
  return x;
}

// Coefficient type of the line sums: FP64 with the FP64 D for FP64 fields;
// for FP32 fields FP32 with the FP32-rounded D up to order kF32SumOrder
// (within the FP32 bound there; FP32 FMAs need no conversions and half the
// registers), FP64 above it.
template <int N, typename T>
using coef_t = typename std::conditional<std::is_same<T, float>::value && f32_line_sums(N),
                                         float, double>::type;

// 1-D contractions at node (i, j, k) of a tile in LDS, line-shifted, summed
// in the coefficient type C.
template <int N, typename T, typename C>
__device__ __forceinline__ void ref_derivs(const T* __restrict__ f,
                                           const C* __restrict__ d, int i, int j, int k,
                                           T& fr, T& fs, T& ft) {
  constexpr int P = N + 1;
  const T* lr = f + (k * P + j) * P;   // line along i
  const T* ls = f + k * P * P + i;     // along j, stride P
  const T* lt = f + j * P + i;         // along k, stride P^2
  const C r0 = lr[0], s0 = ls[0], t0 = lt[0];
  C ar = C(0), as = C(0), at = C(0);
#pragma unroll
  for (int m = 1; m < P; ++m) {
    ar = fma(d[i * P + m], (C)lr[m] - r0, ar);
    as = fma(d[j * P + m], (C)ls[m * P] - s0, as);
    at = fma(d[k * P + m], (C)lt[m * P * P] - t0, at);
  }
  fr = (T)ar;
  fs = (T)as;
  ft = (T)at;
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
  // FP32: the hardware reciprocal (1 ulp) instead of the correctly rounded
  // division sequence, far inside the FP32 bound of the derived fields
  T inv;
  if constexpr (std::is_same<T, float>::value) inv = __builtin_amdgcn_rcpf(det);
  else inv = T(1) / det;
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

// 1 / x from the hardware estimate and two Newton steps (within an ulp or
// two; the correctly rounded division adds range scaling and a final
// correction); x outside [2^-1000, 2^1000] in magnitude, 0 and NaN take the
// division (a branch that a wave skips unless one of its lanes needs it).
__device__ __forceinline__ double recip_refined(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  const double a = fabs(x);
  const bool out = !(a >= 0x1p-1000 && a <= 0x1p+1000);
  if (__builtin_amdgcn_ballot_w64(out) != 0) {   // wave-uniform: skipped as a whole
    double xx = x;
    asm volatile("" : "+v"(xx));   // keeps the division from being hoisted out
    if (out) r = 1.0 / xx;
  }
  return r;
}

// sqrt(x) from the hardware estimate of 1 / sqrt(x), one Goldschmidt step and
// a Newton correction of the root (within an ulp or two); x outside
// [2^-1000, 2^1000], 0 and NaN take the library root.
__device__ __forceinline__ double sqrt_refined(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  double sq = x * r, hr = 0.5 * r;
  const double e = fma(-hr, sq, 0.5);
  sq = fma(sq, e, sq);
  hr = fma(hr, e, hr);
  sq = fma(fma(-sq, sq, x), hr, sq);
  const bool out = !(x >= 0x1p-1000 && x <= 0x1p+1000);
  if (__builtin_amdgcn_ballot_w64(out) != 0) {   // wave-uniform: skipped as a whole
    double xx = x;
    asm volatile("" : "+v"(xx));   // keeps the root from being hoisted out
    if (out) sq = sqrt(xx);
  }
  return sq;
}

// Root of |omega|^2: FP32 takes the hardware square root (v_sqrt_f32, within
// 1 ulp; the correctly rounded form adds range scaling and a correction of
// the last bit, a dozen instructions per node), FP64 the refined estimate
// above.
__device__ __forceinline__ float vort_root(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double vort_root(double x) { return sqrt_refined(x); }

// The adjugate of J (det J times J^-1, same layout as InvJac) and 1 / det J.
__device__ __forceinline__ bool adjugate_jacobian(double xr, double xs, double xt, double yr,
                                                  double ys, double yt, double zr, double zs,
                                                  double zt, InvJac<double>& k, double& inv) {
  k.rx = ys * zt - yt * zs;
  k.sx = yt * zr - yr * zt;
  k.tx = yr * zs - ys * zr;
  const double det = xr * k.rx + xs * k.sx + xt * k.tx;
  inv = recip_refined(det);
  k.ry = xt * zs - xs * zt;
  k.rz = xs * yt - xt * ys;
  k.sy = xr * zt - xt * zr;
  k.sz = xt * yr - xr * yt;
  k.ty = xs * zr - xr * zs;
  k.tz = xr * ys - xs * yr;
  return det > 0.0;
}

// ---------------------------------------------------------------------------
// gradient / Q-criterion: one workgroup per element, tiles staged in LDS
// ---------------------------------------------------------------------------

template <int N, typename T>
__global__ void __launch_bounds__(Shape<N>::kNodeThreads)
derivs_tile(const coef_t<N, T>* __restrict__ dmat, const T* __restrict__ x, const T* __restrict__ y,
            const T* __restrict__ z, const T* __restrict__ f, T* __restrict__ gx,
            T* __restrict__ gy, T* __restrict__ gz, int32_t* __restrict__ status) {
  using S = Shape<N>;
  __shared__ coef_t<N, T> sd[S::P * S::P];
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
__device__ __forceinline__ void qcrit_tile_elem(
    int64_t e, int t, const coef_t<N, T>* __restrict__ dmat, const T* __restrict__ x,
    const T* __restrict__ y, const T* __restrict__ z, const T* __restrict__ u,
    const T* __restrict__ v, const T* __restrict__ w, T* __restrict__ q, T* __restrict__ om,
    T* __restrict__ qmm, int32_t* __restrict__ status) {
  using S = Shape<N>;
  __shared__ coef_t<N, T> sd[S::P * S::P];
  __shared__ T sf[6][S::NP];
  __shared__ T red[2 * (S::kNodeThreads / 64)];
  const int64_t base = e * S::NP;
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
    if (om) om[base + t] = vort_root(w1 * w1 + w2 * w2 + w3 * w3);
    if (qv != qv) qv = neg_inf<T>();
  }
  bad = __syncthreads_or(bad);
  if (bad && t == 0 && status) atomicOr(status, SEM_FLAG_BAD_JACOBIAN);
  if (qmm) {
    T mn = t < S::NP ? qv : pos_inf<T>();
    T mx = qv;
    block_minmax<T, S::kNodeThreads>(mn, mx, red);
    if (t == 0) {
      qmm[2 * e] = mn;
      qmm[2 * e + 1] = mx;
    }
  }
}

template <int N, typename T>
__global__ void __launch_bounds__(Shape<N>::kNodeThreads)
qcrit_tile(const coef_t<N, T>* __restrict__ dmat, const T* __restrict__ x, const T* __restrict__ y,
           const T* __restrict__ z, const T* __restrict__ u, const T* __restrict__ v,
           const T* __restrict__ w, T* __restrict__ q, T* __restrict__ om,
           T* __restrict__ qmm, int32_t* __restrict__ status) {
  qcrit_tile_elem<N, T>(blockIdx.x, threadIdx.x, dmat, x, y, z, u, v, w, q, om, qmm, status);
}

// ---------------------------------------------------------------------------
// gradient / Q-criterion, pencil form: two halves of LT threads per element
// ---------------------------------------------------------------------------
//
// A half is one wave for N <= 7 ((N+1)^2 <= 64 lines) and two waves for
// N = 8, 9.  Thread p < (N+1)^2 of each half owns the r-line
// (j, k) = (p % P, p / P) of the element; half h owns the nodes i in
// [h*H0, h*H0 + H0) of that line, so every node belongs to exactly one
// thread.  Per field:
//   1. each thread loads its whole r-line from HBM (both halves read the
//      same line; the second read hits the cache) and applies D along r for
//      its half -- D entries are uniform across the wave;
//   2. the owners write their nodes to an LDS tile;
//   3. half 0 applies D along s (thread p owns the s-line (i, k)), half 1
//      along t (thread p owns the t-line (i, j)); results go to two LDS
//      tiles;
//   4. the owners read back f_s, f_t at their nodes.
// Each line is read once and each derivative crosses LDS once, instead of
// P LDS reads of the field and P of D per output.  LDS tiles use a padded
// row stride of P + 1.

template <int N, int E = 1>
struct Pen {
  static constexpr int P = N + 1;
  static constexpr int NP = P * P;        // lines per direction and element
  static constexpr int LE = E * NP;       // lines per half (E elements)
  static constexpr int LT = 64 * ((LE + 63) / 64);  // threads per half
  static constexpr int TH = 2 * LT;       // threads per workgroup
  static constexpr int H0 = (P + 1) / 2;  // nodes per thread and half
  static constexpr int RS = P + 1;        // LDS row stride (j)
  static constexpr int SS = P * RS;       // LDS slab stride (k)
  static constexpr int SZ = P * SS;       // padded tile of one element
  static_assert(LE <= LT && TH <= 1024, "one line per thread of a half");
  __device__ static constexpr int at(int i, int j, int k) { return i + RS * j + SS * k; }
  // element of line p (lines of consecutive elements follow each other)
  __device__ static constexpr int elem(int p) { return E == 1 ? 0 : p / NP; }
  // half of thread t, wave-uniform and visibly 0 or 1 (so that the compiler
  // resolves the node-range checks h * H0 + ii < P without branches)
  __device__ static int half(int t) {
    return __builtin_amdgcn_readfirstlane(t >= LT ? 1 : 0) != 0 ? 1 : 0;
  }
};

// Coefficient tables (D, its even-odd halves) are read through the
// constant address space: the index is wave-uniform, so every read is a
// scalar load whatever stores precede it in the kernel.
using const_f64 = const __attribute__((address_space(4))) double*;
using const_f32 = const __attribute__((address_space(4))) float*;
__device__ __forceinline__ double coef(const double* p, int idx) {
  return ((const_f64)p)[idx];
}
__device__ __forceinline__ float coef(const float* p, int idx) {
  return ((const_f32)p)[idx];
}

// Line-shifted derivative of a P-point line: out[i] = sum_m D[i][m] (g_m - g_0),
// summed in the coefficient type C (as ref_derivs).
template <int P, typename T, typename C>
__device__ __forceinline__ T line_deriv(const C* __restrict__ d, int i, const T (&g)[P]) {
  C acc = C(0);
  const C g0 = g[0];
#pragma unroll
  for (int m = 1; m < P; ++m) acc = fma(coef(d, i * P + m), (C)g[m] - g0, acc);
  return (T)acc;
}

// All P outputs of one line (line-shifted as line_deriv) through the
// even-odd halves of D stored after D itself: an output pair (i, P-1-i)
// costs P multiply-adds instead of 2 (P - 1).
template <int P, typename T, typename C>
__device__ __forceinline__ void line_deriv_all(const C* __restrict__ d, const T (&g)[P],
                                               T (&out)[P]) {
  constexpr int H = P / 2, NE = (P + 1) / 2;
  const C* a = d + P * P;
  const C* b = a + NE * NE;
  const C g0 = g[0];
  C hv[P], e[NE], o[H > 0 ? H : 1];
#pragma unroll
  for (int m = 1; m < P; ++m) hv[m] = (C)g[m] - g0;
  // hv[0] = 0: e[0] = hv[P-1], o[0] = -hv[P-1] (written out, since 0 + x
  // does not fold for a possibly negative zero x)
  if constexpr (H > 0) {
    e[0] = hv[P - 1];
    o[0] = -hv[P - 1];
  }
#pragma unroll
  for (int m = 1; m < H; ++m) {
    e[m] = hv[m] + hv[P - 1 - m];
    o[m] = hv[m] - hv[P - 1 - m];
  }
  if constexpr (P % 2 == 1) e[H] = hv[H];   // P odd: H >= 1
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    C pe = coef(a, NE * i) * e[0];
#pragma unroll
    for (int m = 1; m < NE; ++m) pe = fma(coef(a, NE * i + m), e[m], pe);
    C ro = C(0);
    if constexpr (H > 0) ro = coef(b, H * i) * o[0];
#pragma unroll
    for (int m = 1; m < H; ++m) ro = fma(coef(b, H * i + m), o[m], ro);
    out[i] = (T)(ro + pe);
    if (P - 1 - i != i) out[P - 1 - i] = (T)(ro - pe);
  }
}

// One field through the pencil scheme; owner gets (f_r, f_s, f_t) at its
// H0 nodes.  `gf` points at the element's first value.
// Load the owner's r-line of one field (issued early so that several
// fields' loads are in flight at once).
// Line p of a block of elements is the P values at gf + P p; lines from nl
// on (past the last element) are not loaded.
template <int N, typename T>
__device__ __forceinline__ void pencil_load(const T* __restrict__ gf, int p, int nl,
                                            T (&f)[N + 1]) {
  constexpr int P = N + 1;
  if (p < nl) {
#pragma unroll
    for (int m = 0; m < P; ++m) f[m] = gf[p * P + m];
  }
}

template <int N, int E = 1, typename T>
__device__ __forceinline__ void pencil_pass(const T (&f)[N + 1],
                                            const coef_t<N, T>* __restrict__ d,
                                            T* __restrict__ F, T* __restrict__ S,
                                            T* __restrict__ Tt, int h, int p,
                                            T (&fr)[Pen<N>::H0], T (&fs)[Pen<N>::H0],
                                            T (&ft)[Pen<N>::H0]) {
  using Q = Pen<N, E>;
  constexpr int P = Q::P, H0 = Q::H0;
  const bool valid = p < Q::LE;
  const int el = Q::elem(p), line = p - el * Q::NP;
  F += el * Q::SZ;
  S += el * Q::SZ;
  Tt += el * Q::SZ;
  const int j = line % P, k = line / P;
  if (valid) {
#pragma unroll
    for (int ii = 0; ii < H0; ++ii) {
      const int i = h * H0 + ii;
      if (i < P) {
        fr[ii] = line_deriv<P>(d, i, f);
        // f[i] by one select on the wave-uniform half (an index into the
        // line would become a compare-and-select over all P values); at odd
        // P the two values are made opaque first, or the select of two
        // loads is folded into one load at a selected index, which keeps
        // the line in memory
        const T f0 = f[ii], f1 = f[H0 + ii < P ? H0 + ii : P - 1];
        if constexpr (P % 2 == 1) F[Q::at(i, j, k)] = h == 0 ? opaque(f0) : opaque(f1);
        else F[Q::at(i, j, k)] = h == 0 ? f0 : f1;
      }
    }
  }
  __syncthreads();
  if (valid) {
    const int a = j, b = k;
    T g[P], out[P];
    if (h == 0) {  // s-line at (i, k) = (a, b)
#pragma unroll
      for (int m = 0; m < P; ++m) g[m] = F[Q::at(a, m, b)];
      line_deriv_all<P>(d, g, out);
#pragma unroll
      for (int jj = 0; jj < P; ++jj) S[Q::at(a, jj, b)] = out[jj];
    } else {       // t-line at (i, j) = (a, b)
#pragma unroll
      for (int m = 0; m < P; ++m) g[m] = F[Q::at(a, b, m)];
      line_deriv_all<P>(d, g, out);
#pragma unroll
      for (int kk = 0; kk < P; ++kk) Tt[Q::at(a, b, kk)] = out[kk];
    }
  }
  __syncthreads();
  if (valid) {
#pragma unroll
    for (int ii = 0; ii < H0; ++ii) {
      const int i = h * H0 + ii;
      if (i < P) {
        fs[ii] = S[Q::at(i, j, k)];
        ft[ii] = Tt[Q::at(i, j, k)];
      }
    }
  }
}

template <int N, typename T, int E = 1>
struct PencilTiles {
  T F[E * Pen<N>::SZ];
  T S[E * Pen<N>::SZ];
  T Tt[E * Pen<N>::SZ];
  T red[2 * Pen<N, E>::TH / 64];
  int flag;
};

// Geometry of the owner's nodes: J^-1 from the three coordinate passes.
// The coordinate tiles land in FX, FY, FZ (the same tile when they are not
// needed afterwards).
template <int N, int E = 1, typename T>
__device__ __forceinline__ bool pencil_geometry(const T (&lx)[N + 1], const T (&ly)[N + 1],
                                                const T (&lz)[N + 1],
                                                const coef_t<N, T>* __restrict__ d,
                                                PencilTiles<N, T, E>& sm, T* FX, T* FY, T* FZ,
                                                int h, int p, InvJac<T> (&kk)[Pen<N>::H0]) {
  constexpr int H0 = Pen<N>::H0, P = Pen<N>::P;
  T xr[H0], xs[H0], xt[H0], yr[H0], ys[H0], yt[H0], zr[H0], zs[H0], zt[H0];
  pencil_pass<N, E>(lx, d, FX, sm.S, sm.Tt, h, p, xr, xs, xt);
  pencil_pass<N, E>(ly, d, FY, sm.S, sm.Tt, h, p, yr, ys, yt);
  pencil_pass<N, E>(lz, d, FZ, sm.S, sm.Tt, h, p, zr, zs, zt);
  bool ok = true;
#pragma unroll
  for (int ii = 0; ii < H0; ++ii) {
    const bool good = invert_jacobian(xr[ii], xs[ii], xt[ii], yr[ii], ys[ii], yt[ii], zr[ii],
                                      zs[ii], zt[ii], kk[ii]);
    if (h * H0 + ii < P) ok = ok && good;   // odd P: half 1 owns one node fewer
  }
  return ok;
}

template <int N, typename T>
__global__ void __launch_bounds__(Pen<N>::TH)
derivs_pencil(const coef_t<N, T>* __restrict__ dmat, const T* __restrict__ x, const T* __restrict__ y,
              const T* __restrict__ z, const T* __restrict__ f, T* __restrict__ gx,
              T* __restrict__ gy, T* __restrict__ gz, int32_t* __restrict__ status) {
  using Q = Pen<N>;
  constexpr int P = Q::P, H0 = Q::H0;
  __shared__ PencilTiles<N, T> sm;
  const int h = Q::half(threadIdx.x);
  const int p = threadIdx.x % Q::LT;
  const int64_t base = (int64_t)blockIdx.x * (P * P * P);
  T lx[P], ly[P], lz[P], lf[P];
  pencil_load<N>(x + base, p, Q::NP, lx);
  pencil_load<N>(y + base, p, Q::NP, ly);
  pencil_load<N>(z + base, p, Q::NP, lz);
  pencil_load<N>(f + base, p, Q::NP, lf);
  InvJac<T> kk[H0];
  int bad = !pencil_geometry<N>(lx, ly, lz, dmat, sm, sm.F, sm.F, sm.F, h, p, kk);
  T fr[H0], fs[H0], ft[H0];
  pencil_pass<N>(lf, dmat, sm.F, sm.S, sm.Tt, h, p, fr, fs, ft);
  const bool valid = p < Q::NP;
  if (!valid) bad = 0;
  if (valid) {
    const int j = p % P, k = p / P;
#pragma unroll
    for (int ii = 0; ii < H0; ++ii) {
      const int i = h * H0 + ii;
      if (i < P) {
        const int64_t o = base + (k * P + j) * P + i;
        gx[o] = fr[ii] * kk[ii].rx + fs[ii] * kk[ii].sx + ft[ii] * kk[ii].tx;
        gy[o] = fr[ii] * kk[ii].ry + fs[ii] * kk[ii].sy + ft[ii] * kk[ii].ty;
        gz[o] = fr[ii] * kk[ii].rz + fs[ii] * kk[ii].sz + ft[ii] * kk[ii].tz;
      }
    }
  }
  bad = __syncthreads_or(bad);
  if (bad && threadIdx.x == 0 && status) atomicOr(status, SEM_FLAG_BAD_JACOBIAN);
}

// Q and |omega| at the owner's nodes; the velocity-gradient rows are folded
// into Q = -(sum_ij A_ij A_ji)/2 and |omega|^2 as they are produced.
template <int N, int E = 1, typename T>
__device__ __forceinline__ bool pencil_qcrit(const T* gx, const T* gy, const T* gz,
                                             const T* gu, const T* gv, const T* gw,
                                             const coef_t<N, T>* __restrict__ d,
                                             PencilTiles<N, T, E>& sm, T* FX, T* FY, T* FZ,
                                             int h, int p, int nl, T (&qv)[Pen<N>::H0],
                                             T (&om)[Pen<N>::H0]) {
  constexpr int H0 = Pen<N>::H0, P = Pen<N>::P;
  // N <= 7 and FP32: all six lines are requested before any arithmetic;
  // FP64 at N = 8, 9: the velocity lines are requested just before their
  // pass (their values would otherwise hold 60 more registers through the
  // geometry). FP32 at N = 9 stays at 187 registers either way, and the
  // early requests took its Q phase on the batch benchmark's order-9
  // snapshots from 3.96 to 3.64 ms.
  constexpr bool kEarly = N <= 7 || std::is_same<T, float>::value;
  T lx[P], ly[P], lz[P], lu[P], lv[P], lw[P];
  pencil_load<N>(gx, p, nl, lx);
  pencil_load<N>(gy, p, nl, ly);
  pencil_load<N>(gz, p, nl, lz);
  if constexpr (kEarly) {
    pencil_load<N>(gu, p, nl, lu);
    pencil_load<N>(gv, p, nl, lv);
    pencil_load<N>(gw, p, nl, lw);
  }
  InvJac<T> kk[H0];
  const bool ok = pencil_geometry<N, E>(lx, ly, lz, d, sm, FX, FY, FZ, h, p, kk);
  T fr[H0], fs[H0], ft[H0];
  T a01[H0], a02[H0], a12[H0];
  // row 0 (u)
  if constexpr (!kEarly) pencil_load<N>(gu, p, nl, lu);
  pencil_pass<N, E>(lu, d, sm.F, sm.S, sm.Tt, h, p, fr, fs, ft);
#pragma unroll
  for (int ii = 0; ii < H0; ++ii) {
    const InvJac<T>& K = kk[ii];
    const T a00 = fr[ii] * K.rx + fs[ii] * K.sx + ft[ii] * K.tx;
    a01[ii] = fr[ii] * K.ry + fs[ii] * K.sy + ft[ii] * K.ty;
    a02[ii] = fr[ii] * K.rz + fs[ii] * K.sz + ft[ii] * K.tz;
    qv[ii] = a00 * a00;
  }
  // row 1 (v)
  if constexpr (!kEarly) pencil_load<N>(gv, p, nl, lv);
  pencil_pass<N, E>(lv, d, sm.F, sm.S, sm.Tt, h, p, fr, fs, ft);
#pragma unroll
  for (int ii = 0; ii < H0; ++ii) {
    const InvJac<T>& K = kk[ii];
    const T a10 = fr[ii] * K.rx + fs[ii] * K.sx + ft[ii] * K.tx;
    const T a11 = fr[ii] * K.ry + fs[ii] * K.sy + ft[ii] * K.ty;
    a12[ii] = fr[ii] * K.rz + fs[ii] * K.sz + ft[ii] * K.tz;
    qv[ii] = qv[ii] + a11 * a11 + T(2) * (a01[ii] * a10);
    const T w3 = a10 - a01[ii];
    om[ii] = w3 * w3;
  }
  // row 2 (w)
  if constexpr (!kEarly) pencil_load<N>(gw, p, nl, lw);
  pencil_pass<N, E>(lw, d, sm.F, sm.S, sm.Tt, h, p, fr, fs, ft);
#pragma unroll
  for (int ii = 0; ii < H0; ++ii) {
    const InvJac<T>& K = kk[ii];
    const T a20 = fr[ii] * K.rx + fs[ii] * K.sx + ft[ii] * K.tx;
    const T a21 = fr[ii] * K.ry + fs[ii] * K.sy + ft[ii] * K.ty;
    const T a22 = fr[ii] * K.rz + fs[ii] * K.sz + ft[ii] * K.tz;
    qv[ii] = T(-0.5) * (qv[ii] + a22 * a22 + T(2) * (a02[ii] * a20 + a12[ii] * a21));
    const T w1 = a21 - a12[ii], w2 = a02[ii] - a20;
    om[ii] = vort_root(om[ii] + w1 * w1 + w2 * w2);
  }
  return ok;
}

// Counting four isovalues at a time. A node's word holds bit (q > c_s) at
// bit 8s for the isovalues g .. g + 3 below n (a NaN compares below every
// isovalue); the eight corner words of a cell, each shifted by its vertex
// number (vertex bits x, y, z = 1, 2, 4) and summed, hold the cell's four
// cases as bytes. A case maps to triangles + (1 << 16) when non-trivial, so
// one sum per isovalue gives both the triangle and the active-cell count.
template <typename T>
__device__ __forceinline__ uint32_t iso_bits4(T q, const IsoList<T>& iso, int g, int n) {
  uint32_t b = 0;
#pragma unroll
  for (int s = 0; s < 4; ++s)
    if (g + s < n) b |= (uint32_t)(q > iso.v[g + s]) << (8 * s);
  return b;
}
template <int RS, int SS>
__device__ __forceinline__ uint32_t cell_word(const uint32_t* bits, int n0) {
  uint32_t w = 0;
#pragma unroll
  for (int vtx = 0; vtx < 8; ++vtx)
    w += bits[n0 + (vtx & 1) + RS * ((vtx >> 1) & 1) + SS * (vtx >> 2)] << vtx;
  return w;
}
__device__ __forceinline__ int case_count_entry(int cs, uint8_t nt) {
  return (int)nt + ((cs != 0 && cs != 255) << 16);
}
// Sum over the 16 lanes of each row of the wave, by DPP row shifts (lanes
// shifted in from outside the row read 0): lane 15 of the row ends with the
// row's sum (the others with partial sums).  Four VALU operations, no LDS.
__device__ __forceinline__ uint32_t row_sum16(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);   // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);   // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);   // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);   // row_shr:8
  return v;
}

// Sum over the wave, left in lane 63 (other lanes hold partial sums): the
// row sums above, then lane 15 of rows 0 and 2 added into rows 1 and 3
// (row_bcast:15) and lane 31 into rows 2 and 3 (row_bcast:31); lanes of the
// rows a row mask leaves out add 0.  Every lane of the wave must be active.
__device__ __forceinline__ uint32_t wave_sum_to63(uint32_t v) {
  v = row_sum16(v);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// Order-7 cell c = i + 7 j + 49 k has corner 0 at node i + 8 j + 64 k =
// c + c / 7 + 8 (c / 49); the divisions by multiply and shift, exact for
// c < 512 (the rounding errors stay below the gap to the next integer).
__device__ __forceinline__ int cell_base7(int c) {
  return c + ((c * 9363) >> 16) + 8 * ((c * 1338) >> 16);
}

// Case-table entry for packed counting: triangles + (1 << 8) for a
// non-trivial case.
__device__ __forceinline__ int case_count_entry8(int cs, uint8_t nt) {
  return (int)nt + ((cs != 0 && cs != 255) << 8);
}

// Element counts of the isovalues g .. g + m - 1 (m <= 4) for a workgroup
// of NW <= 4 waves with at most three cells per lane: pw[s >> 1] holds, in
// its 16-bit half s & 1, the lane's triangles + (active cells << 8) of
// isovalue s (at most 3 x 5 triangles per lane, so a row of 16 lanes stays
// below 240 + (48 << 8)).  DPP row sums, the 4 NW row sums through s_rows
// (8 NW words), one barrier, then wave 0 sums the rows of each isovalue.
// s_rows must not be written again before a later barrier.
template <int NW>
__device__ __forceinline__ void publish_rows(uint32_t (&pw)[2], int m, int g, int t,
                                             uint32_t* s_rows, int32_t* __restrict__ cnt,
                                             int64_t n_elem, int64_t e,
                                             int64_t* __restrict__ active) {
  static_assert(NW >= 1 && NW <= 4, "at most 16 rows");
  const int h = t >> 6, p = t & 63;
  pw[0] = row_sum16(pw[0]);
  if (m > 2) pw[1] = row_sum16(pw[1]);
  if ((p & 15) == 15) {
    s_rows[2 * (4 * h + (p >> 4))] = pw[0];
    s_rows[2 * (4 * h + (p >> 4)) + 1] = pw[1];
  }
  __syncthreads();
  if (h == 0) {
    const int row = p & 15, s = p >> 4;   // lane: one row's field of isovalue s
    const uint32_t f =
        row < 4 * NW ? (s_rows[2 * row + (s >> 1)] >> (16 * (s & 1))) & 0xffffu : 0u;
    const uint32_t sum = row_sum16((f & 255u) | ((f >> 8) << 16));
    if (row == 15 && s < m) {
      cnt[(int64_t)(g + s) * n_elem + e] = (int)(sum & 0xffffu);
      const unsigned a = sum >> 16;
      if (active && a) atomicAdd((unsigned long long*)&active[g + s], (unsigned long long)a);
    }
  }
}
// Where a Q kernel also counts each isovalue's triangles and active cells per
// element (the count pass of the isosurface, fused).
template <typename T>
struct CountSink {
  int n_iso;
  IsoList<T> iso;
  const uint8_t* ntri;     // [256] triangles per case
  int32_t* cnt;            // [n_iso][n_elem]
  int64_t* active;         // [n_iso] active-cell totals (may be NULL)
  int64_t n_elem;
};

// Ranges and counts of a workgroup of E > 1 elements: wave w takes the
// elements w, w + waves, ...; an element's range from its lines' partial
// (min, max) in part (both halves), its cells' cases from the node words in
// F (one element tile after another).
template <int N, typename T, bool COUNT, int E>
__device__ __forceinline__ void pencil_multi_tail(int64_t e, int t, int ne,
                                                  const T (&qv)[Pen<N>::H0], T* F,
                                                  const T* part, T* emm, const int32_t* tab,
                                                  T* __restrict__ qmm,
                                                  const CountSink<T>* sink) {
  using Q = Pen<N, E>;
  constexpr int P = Q::P, H0 = Q::H0, NW = Q::TH / 64;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;
  for (int el = wave; el < ne; el += NW) {
    T a = pos_inf<T>(), b = neg_inf<T>();
    for (int q2 = lane; q2 < 2 * Q::NP; q2 += 64) {
      const int idx = (q2 < Q::NP ? 0 : Q::LT - Q::NP) + el * Q::NP + q2;
      a = part[idx] < a ? part[idx] : a;
      b = part[Q::TH + idx] > b ? part[Q::TH + idx] : b;
    }
    wave_minmax(a, b);
    if (lane == 63) {
      if (qmm) {
        qmm[2 * (e + el)] = a;
        qmm[2 * (e + el) + 1] = b;
      }
      if constexpr (COUNT) {
        emm[2 * el] = a;
        emm[2 * el + 1] = b;
      }
    }
  }
  if constexpr (COUNT) {
    constexpr int NC = N * N * N;
    uint32_t* bits = reinterpret_cast<uint32_t*>(F);
    const int h = Q::half(t);
    const int p = t % Q::LT;
    const bool valid = p < ne * Q::NP;
    const int n_iso = sink->n_iso;
    __syncthreads();   // publishes emm
    for (int g = 0; g < n_iso; g += 4) {
      const int m = n_iso - g < 4 ? n_iso - g : 4;
      if (g > 0) {
        __syncthreads();   // every wave is done with the previous words
        if (valid) {
          const int el = Q::elem(p), line = p - el * Q::NP;
          const int j = line % P, k = line / P;
#pragma unroll
          for (int ii = 0; ii < H0; ++ii) {
            const int i = h * H0 + ii;
            if (i < P)
              bits[el * Q::SZ + Q::at(i, j, k)] = iso_bits4<T>(qv[ii], sink->iso, g, n_iso);
          }
        }
        __syncthreads();
      }
      for (int el = wave; el < ne; el += NW) {
        // elements outside every isovalue's range of the group have only
        // trivial cases (NaN nodes count as below; the minimum is -inf then)
        const T emn = emm[2 * el], emx = emm[2 * el + 1];
        bool live = false;
        for (int s = 0; s < m; ++s)
          live |= (emx > sink->iso.v[g + s]) && !(emn > sink->iso.v[g + s]);
        int packed[4] = {0, 0, 0, 0};
        if (live) {
          for (int c = lane; c < NC; c += 64) {
            const int n0 = el * Q::SZ + Q::at(c % N, (c / N) % N, c / (N * N));
            const uint32_t word = cell_word<Q::RS, Q::SS>(bits, n0);
#pragma unroll
            for (int s = 0; s < 4; ++s)
              if (s < m) packed[s] += tab[(word >> (8 * s)) & 255];
          }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          if (s < m) {
            const int sum = (int)wave_sum_to63((uint32_t)packed[s]);
            if (lane == 63) {
              sink->cnt[(int64_t)(g + s) * sink->n_elem + e + el] = sum & 0xffff;
              const int a = sum >> 16;
              if (sink->active && a)
                atomicAdd((unsigned long long*)&sink->active[g + s], (unsigned long long)a);
            }
          }
        }
      }
    }
  }
}

// One workgroup over the elements e .. e + ne - 1 (E of them at most).
template <int N, typename T, bool COUNT = false, int E = 1>
__device__ __forceinline__ void qcrit_pencil_elem(
    int64_t e, int t, const coef_t<N, T>* __restrict__ dmat, const T* __restrict__ x,
    const T* __restrict__ y, const T* __restrict__ z, const T* __restrict__ u,
    const T* __restrict__ v, const T* __restrict__ w, T* __restrict__ q, T* __restrict__ om,
    T* __restrict__ qmm, int32_t* __restrict__ status, const CountSink<T>* sink = nullptr,
    int ne = 1) {
  using Q = Pen<N, E>;
  constexpr int P = Q::P, H0 = Q::H0;
  __shared__ PencilTiles<N, T, E> sm;
  __shared__ int32_t s_tab[COUNT ? 256 : 1];
  __shared__ uint32_t s_rows[COUNT && E == 1 ? 2 * Q::TH / 64 * 4 : 1];
  __shared__ T s_part[E > 1 ? 2 * Q::TH : 1];   // per-thread (min, max) of Q
  __shared__ T s_emm[E > 1 && COUNT ? 2 * E : 1];
  const int h = Q::half(t);
  const int p = t % Q::LT;
  const int64_t base = e * (P * P * P);
  const int nl = E == 1 ? Q::NP : ne * Q::NP;   // lines of elements that exist
  // triangle counts of the 256 cases: requested here, written to LDS after
  // the passes (published by the barrier after the Q tile), so that the
  // loads overlap the field loads instead of delaying them
  constexpr int TR = COUNT ? (256 + Q::TH - 1) / Q::TH : 1;
  uint8_t tab_v[TR];
  if constexpr (COUNT) {
#pragma unroll
    for (int r = 0; r < TR; ++r)
      if (t + r * Q::TH < 256) tab_v[r] = sink->ntri[t + r * Q::TH];
  }
  T qv[H0], ov[H0];
  int bad = !pencil_qcrit<N, E>(x + base, y + base, z + base, u + base, v + base, w + base,
                                dmat, sm, sm.F, sm.F, sm.F, h, p, nl, qv, ov);
  if constexpr (COUNT) {
    // the several-element tail packs active cells at bit 16, the
    // one-element form at bit 8
#pragma unroll
    for (int r = 0; r < TR; ++r) {
      const int c = t + r * Q::TH;
      if (c < 256) s_tab[c] = E == 1 ? case_count_entry8(c, tab_v[r]) : case_count_entry(c, tab_v[r]);
    }
  }
  const bool valid = p < nl;
  T mn = pos_inf<T>(), mx = neg_inf<T>();
  if (!valid) bad = 0;
  if (valid) {
    const int el = Q::elem(p), line = p - el * Q::NP;
    const int j = line % P, k = line / P;
#pragma unroll
    for (int ii = 0; ii < H0; ++ii) {
      const int i = h * H0 + ii;
      if (i < P) {
        const int64_t o = base + (int64_t)p * P + i;   // line p of the block, node i
        if (q) q[o] = qv[ii];
        if (om) om[o] = ov[ii];
        if constexpr (COUNT)   // F is free after the last pass
          reinterpret_cast<uint32_t*>(sm.F)[el * Q::SZ + Q::at(i, j, k)] =
              iso_bits4<T>(qv[ii], sink->iso, 0, sink->n_iso);
        const T c = qv[ii] != qv[ii] ? neg_inf<T>() : qv[ii];
        mn = c < mn ? c : mn;
        mx = c > mx ? c : mx;
      }
    }
  }
  if constexpr (E > 1) {
    s_part[t] = mn;
    s_part[Q::TH + t] = mx;
  }
  // an inverted element (rare) is flagged by its own lanes: no block vote
  if (bad && status) atomicOr(status, SEM_FLAG_BAD_JACOBIAN);
  __syncthreads();               // publishes the Q tile
  if constexpr (E > 1) {
    pencil_multi_tail<N, T, COUNT, E>(e, t, ne, qv, sm.F, s_part, s_emm, s_tab, qmm, sink);
    return;
  }
  if (qmm || COUNT) {
    block_minmax<T, Q::TH>(mn, mx, sm.red);
    if (qmm && t == 0) {
      qmm[2 * e] = mn;
      qmm[2 * e + 1] = mx;
    }
  }
  if constexpr (COUNT && E == 1) {
    // cells t, t + TH, ...; node words in F
    constexpr int NC = N * N * N, R = (NC + Q::TH - 1) / Q::TH, NW = Q::TH / 64;
    uint32_t* bits = reinterpret_cast<uint32_t*>(sm.F);
    static_assert(R <= 3, "publish_rows takes at most three cells per lane");
    int n0[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int cc = t + r * Q::TH < NC ? t + r * Q::TH : 0;
      n0[r] = Q::at(cc % N, (cc / N) % N, cc / (N * N));
    }
    const int n_iso = sink->n_iso;
    for (int g = 0; g < n_iso; g += 4) {
      const int m = n_iso - g < 4 ? n_iso - g : 4;
      if (g > 0) {   // every read of the previous words is behind the last barrier
        if (valid) {
          const int j = p % P, k = p / P;
#pragma unroll
          for (int ii = 0; ii < H0; ++ii) {
            const int i = h * H0 + ii;
            if (i < P) bits[Q::at(i, j, k)] = iso_bits4<T>(qv[ii], sink->iso, g, n_iso);
          }
        }
        __syncthreads();
      }
      // elements outside every isovalue's range of the group have only
      // trivial cases (NaN nodes count as below; mn is -inf then)
      bool live = false;
      for (int s = 0; s < m; ++s)
        live |= (mx > sink->iso.v[g + s]) && !(mn > sink->iso.v[g + s]);
      uint32_t pw[2] = {0u, 0u};
      if (live) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (t + r * Q::TH >= NC) continue;
          const uint32_t word = cell_word<Q::RS, Q::SS>(bits, n0[r]);
#pragma unroll
          for (int s = 0; s < 4; ++s)
            if (s < m) pw[s >> 1] += (uint32_t)s_tab[(word >> (8 * s)) & 255] << (16 * (s & 1));
        }
      }
      publish_rows<NW>(pw, m, g, t, s_rows, sink->cnt, sink->n_elem, e, sink->active);
    }
  }
}

// Elements per workgroup of the pencil Q kernels: enough that the lines of
// the low orders fill whole waves ((N + 1)^2 lines per element and half).
// FP32 N = 6 and 8 stay at one: there the larger workgroup costs a wave of
// occupancy per SIMD (143 and 129 registers) and measured slower (34.2
// against 26.6 and 26.0 against 25.4 ps per point). FP64 N = 5, 6 (over 200
// registers) keep workgroups of at most four waves: with eight, the batched
// kernel's registers spill.
constexpr int pencil_elems_of(int n, bool f64) {
  constexpr int e64[kMaxOrder + 1] = {1, 16, 7, 4, 5, 3, 1, 1, 1, 1};
  constexpr int e32[kMaxOrder + 1] = {1, 16, 7, 4, 5, 7, 1, 1, 1, 1};
  return f64 ? e64[n] : e32[n];
}
template <int N, typename T>
constexpr int pencil_elems() {
  return pencil_elems_of(N, std::is_same<T, double>::value);
}
template <int N, typename T>
constexpr int pencil_threads() {
  return Pen<N, pencil_elems<N, T>()>::TH;
}

template <int N, typename T>
__global__ void __launch_bounds__((pencil_threads<N, T>()))
qcrit_pencil(const coef_t<N, T>* __restrict__ dmat, const T* __restrict__ x, const T* __restrict__ y,
             const T* __restrict__ z, const T* __restrict__ u, const T* __restrict__ v,
             const T* __restrict__ w, T* __restrict__ q, T* __restrict__ om,
             T* __restrict__ qmm, int32_t* __restrict__ status, int64_t n_elem) {
  constexpr int E = pencil_elems<N, T>();
  const int64_t e0 = (int64_t)blockIdx.x * E;
  const int ne = n_elem - e0 < E ? (int)(n_elem - e0) : E;
  qcrit_pencil_elem<N, T, false, E>(e0, threadIdx.x, dmat, x, y, z, u, v, w, q, om, qmm,
                                    status, nullptr, ne);
}

// Q, |omega|, range and the per-(isovalue, element) counts in one pass.
template <int N, typename T>
__global__ void __launch_bounds__((pencil_threads<N, T>()))
qcount_pencil(const coef_t<N, T>* __restrict__ dmat, const T* __restrict__ x,
              const T* __restrict__ y, const T* __restrict__ z, const T* __restrict__ u,
              const T* __restrict__ v, const T* __restrict__ w, T* __restrict__ q,
              T* __restrict__ om, T* __restrict__ qmm, int32_t* __restrict__ status,
              CountSink<T> sink) {
  constexpr int E = pencil_elems<N, T>();
  const int64_t e0 = (int64_t)blockIdx.x * E;
  const int ne = sink.n_elem - e0 < E ? (int)(sink.n_elem - e0) : E;
  qcrit_pencil_elem<N, T, true, E>(e0, threadIdx.x, dmat, x, y, z, u, v, w, q, om, qmm,
                                   status, &sink, ne);
}

// ---------------------------------------------------------------------------
// N = 7, FP64: element tiles staged in LDS by direct global->LDS loads
// ---------------------------------------------------------------------------
//
// Each element's six tiles (4 KiB each) are fetched with global_load_lds
// (16 bytes per lane, 1 KiB per wave instruction, fully coalesced, no
// registers held while the data is in flight).  A lane may fetch any
// 16-byte chunk (two neighbouring i) and it lands at LDS slot
// base + lane, so the chunk placement is chosen freely:
//   slot(k, j, ip) = 4 (8k + (j ^ (k & 1))) + (ip ^ ((j >> 1) & 3)),
// i.e. rows j <-> j^1 swapped in odd slabs and the four chunks of a row
// rotated by j >> 1.  With 32 four-byte banks this makes the r-line reads
// (16 bytes per lane, fixed chunk, lanes over j), the s-line reads (8 bytes,
// lanes over i and a pair of k) and the t-line reads (8 bytes, lanes over i
// and a pair of j) free of bank conflicts.

namespace dma7 {
__device__ __forceinline__ constexpr int slot(int k, int j, int ip) {
  return 4 * (8 * k + (j ^ (k & 1))) + (ip ^ ((j >> 1) & 3));
}
__device__ __forceinline__ constexpr int at(int i, int j, int k) {
  return 2 * slot(k, j, i >> 1) + (i & 1);
}
}  // namespace dma7

struct DmaNode {
  __device__ __forceinline__ int operator()(int i, int j, int k) const {
    return dma7::at(i, j, k);
  }
};

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// One 16-byte direct load per lane into LDS at lds + 16 * lane, issued as
// inline assembly: the compiler then keeps no record of the LDS write and
// inserts no waits of its own for it (after LDS lowering it cannot tell the
// tiles apart and would wait for every load in flight before any tile
// read).  Every consumer waits explicitly (s_waitcnt on vmcnt, then a
// barrier) before reading the tile.
__device__ __forceinline__ void lds_load16(const double* src, double* lds) {
  const uint32_t m0 =
      __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_ptr_t)lds);
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
               :
               : "v"(src), "s"(m0)
               : "memory", "m0");
}

// Fetch one 4 KiB tile: wave h issues the chunk groups h and h + 2.
__device__ __forceinline__ void dma_tile(const double* __restrict__ src, double* raw, int h,
                                         int lane) {
#pragma unroll
  for (int pp = 0; pp < 2; ++pp) {
    const int part = 2 * pp + h;
    const int s = 64 * part + lane;
    const int row = s >> 2, k = row >> 3, j = (row & 7) ^ (k & 1);
    const int ip = (s & 3) ^ ((j >> 1) & 3);
    lds_load16(src + 2 * (ip + 4 * j + 32 * k), raw + 128 * part);
  }
}

// s_waitcnt immediate (vmcnt in bits 3:0 and 15:14, expcnt at its maximum,
// lgkmcnt 0): wait until at most n vector-memory operations and no LDS
// operation of this wave are outstanding.
constexpr int waitcnt_vm_lds(int n) { return (n & 15) | ((n >> 4) << 14) | 0x70; }

// Barrier after an explicit wait: a plain s_barrier (the compiler-level
// memory clobbers keep LDS accesses on their side of it).  __syncthreads()
// would add a workgroup fence, which must also wait for every direct load
// still in flight.
__device__ __forceinline__ void barrier_after_wait() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Workgroup barrier for ordinary LDS traffic while direct loads may still be
// in flight: wait for this wave's LDS operations only, then s_barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt and expcnt untouched
  barrier_after_wait();
}

// ---------------------------------------------------------------------------
// marching cubes
// ---------------------------------------------------------------------------

// low corner and axis of each cube edge (edge id = 4*axis + rank)
// Low corner of edge e, packed as 4-bit fields (edge 0 lowest): edges
// 0..3 run along r from corners 0, 2, 4, 6; edges 4..7 along s from 0, 1,
// 4, 5; edges 8..11 along t from 0, 1, 2, 3.  The axis is e >> 2.  Decoded
// with a shift instead of a table, so the vertex loop reads no memory for it.
constexpr uint64_t kEdgeLoPacked = 0x321054106420ull;
__device__ __forceinline__ int edge_lo(int e) { return (int)((kEdgeLoPacked >> (4 * e)) & 15); }

// Node offset of cube corner v in a tile with row stride RS and slab stride SS.
template <int RS, int SS>
__device__ __forceinline__ int corner_offset(int v) {
  return (v & 1) + RS * ((v >> 1) & 1) + SS * ((v >> 2) & 1);
}
template <int P>
__device__ __forceinline__ int corner_offset(int v) {
  return corner_offset<P, P * P>(v);
}

// Case index of the cell whose lowest node sits at tile offset n0.
template <int RS, int SS, typename T>
__device__ __forceinline__ int cell_case_strided(const T* __restrict__ sf, int n0, T c) {
  int cs = 0;
#pragma unroll
  for (int vtx = 0; vtx < 8; ++vtx) cs |= (sf[n0 + corner_offset<RS, SS>(vtx)] > c) << vtx;
  return cs;
}
template <int N, typename T>
__device__ __forceinline__ int cell_case(const T* __restrict__ sf, int n0, T c) {
  return cell_case_strided<N + 1, (N + 1) * (N + 1)>(sf, n0, c);
}

// Exclusive prefix over the cells of a block of the per-cell triangle counts
// nt (0..7): one ballot per bit gives the wave prefix; wave totals go through
// LDS.  Returns the thread's offset; *block_total receives the block total.
template <int TH>
__device__ __forceinline__ int block_count_prefix(int nt, int32_t* s_wave, int* block_total) {
  constexpr int W = TH / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t m0 = __ballot(nt & 1), m1 = __ballot(nt & 2), m2 = __ballot(nt & 4);
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  int pre = __popcll(m0 & lt) + 2 * __popcll(m1 & lt) + 4 * __popcll(m2 & lt);
  if (lane == 0) s_wave[wv] = __popcll(m0) + 2 * __popcll(m1) + 4 * __popcll(m2);
  __syncthreads();
  int tot = 0;
#pragma unroll
  for (int q = 0; q < W; ++q) {
    pre += q < wv ? s_wave[q] : 0;
    tot += s_wave[q];
  }
  __syncthreads();
  *block_total = tot;
  return pre;
}

// Balanced emission of one element's triangles for one isovalue.  First
// every cell (in rounds of TH threads, cell order) records its case and
// writes one descriptor (cell << 3 | slot) per triangle into `desc` at its
// running prefix; then thread v computes vertex v of that list.  Every lane
// does the same amount of work however unevenly the triangles fall on the
// cells, and consecutive lanes write consecutive vertices.  `node(i, j, k)`
// maps a node to its index in the field tile ft, `cnode(i, j, k)` to its
// index in the coordinate arrays sx, sy, sz (a tile in LDS, or the
// element's values in global memory).  Returns the element's triangle count.
template <int N, int TH, typename T, class NodeFn, class CoordFn>
__device__ __forceinline__ int emit_element(T c, NodeFn node, CoordFn cnode,
                                            const T* __restrict__ ft,
                                            const T* __restrict__ sx, const T* __restrict__ sy,
                                            const T* __restrict__ sz,
                                            const uint8_t* __restrict__ s_ntri,
                                            const int8_t* __restrict__ s_tri,
                                            uint8_t* __restrict__ cases,
                                            uint16_t* __restrict__ desc, int32_t* s_wave,
                                            T* __restrict__ out, int64_t g0, int64_t cap,
                                            uint64_t* __restrict__ keys, int64_t key_base) {
  constexpr int P = N + 1, NC = N * N * N, ROUNDS = (NC + TH - 1) / TH;
  const int t = threadIdx.x;
  int run = 0;
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    const int cell = r * TH + t;
    int cs = 0, nt = 0;
    if (cell < NC) {
      const int ci = cell % N, cj = (cell / N) % N, ck = cell / (N * N);
#pragma unroll
      for (int vtx = 0; vtx < 8; ++vtx)
        cs |= (ft[node(ci + (vtx & 1), cj + ((vtx >> 1) & 1), ck + (vtx >> 2))] > c) << vtx;
      nt = s_ntri[cs];
      cases[cell] = (uint8_t)cs;
    }
    int tot;
    const int pre = block_count_prefix<TH>(nt, s_wave, &tot);
    for (int sl = 0; sl < nt; ++sl) desc[run + pre + sl] = (uint16_t)((cell << 3) | sl);
    run += tot;
  }
  __syncthreads();
  for (int vv = t; vv < 3 * run; vv += TH) {
    const int tri = vv / 3, vtx = vv - 3 * tri;
    const int64_t g = g0 + tri;
    if (g >= cap) continue;
    const int dsc = desc[tri];
    const int cell = dsc >> 3, slot = dsc & 7;
    const int cs = cases[cell];
    const int ci = cell % N, cj = (cell / N) % N, ck = cell / (N * N);
    const int edge = s_tri[(cs * kMcMaxTri + slot) * 3 + vtx];
    const int v0 = edge_lo(edge);
    const int ax = edge >> 2;
    const int a0 = ci + (v0 & 1), b0 = cj + ((v0 >> 1) & 1), c0 = ck + (v0 >> 2);
    const int a1 = a0 + (ax == 0), b1 = b0 + (ax == 1), c1 = c0 + (ax == 2);
    const int lo = node(a0, b0, c0), hi = node(a1, b1, c1);
    const int clo = cnode(a0, b0, c0), chi = cnode(a1, b1, c1);
    T* o = out + g * 9 + 3 * vtx;
    {
#pragma clang fp contract(off)
      const T f0 = ft[lo], f1 = ft[hi];
      const T tt = (c - f0) / (f1 - f0);
      o[0] = sx[clo] + tt * (sx[chi] - sx[clo]);
      o[1] = sy[clo] + tt * (sy[chi] - sy[clo]);
      o[2] = sz[clo] + tt * (sz[chi] - sz[clo]);
    }
    if (keys)
      keys[g * 3 + vtx] = (uint64_t)(key_base + a0 + P * (b0 + P * c0)) * 3u + (uint64_t)ax;
  }
  __syncthreads();
  return run;
}

// Tile index functions for emit_element.
template <int RS, int SS>
struct StridedNode {
  __device__ __forceinline__ int operator()(int i, int j, int k) const {
    return i + RS * j + SS * k;
  }
};

// Per (isovalue, element): triangle and active-cell counts; optional case dump.
template <int N, typename T>
__global__ void __launch_bounds__(Shape<N>::kCellThreads)
iso_count(int64_t n_elem, const T* __restrict__ field, const T* __restrict__ mm, int n_iso,
          IsoList<T> iso, const uint8_t* __restrict__ ntri_tab, int32_t* __restrict__ cnt,
          int64_t* __restrict__ active_total, uint8_t* __restrict__ case_idx) {
  using S = Shape<N>;
  constexpr int TH = S::kCellThreads;
  __shared__ T sf[S::NP];
  __shared__ uint32_t s_ntri4[64];
  __shared__ T red[2 * (TH / 64)];
  __shared__ int32_t sred[TH / 64];
  const int t = threadIdx.x;
  const int64_t e = blockIdx.x;
  const int64_t base = e * S::NP;
  const uint8_t* s_ntri = reinterpret_cast<const uint8_t*>(s_ntri4);
  if (t < 64) s_ntri4[t] = reinterpret_cast<const uint32_t*>(ntri_tab)[t];
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
    // triangles in the low 16 bits, active cells above: one block sum
    int packed = 0;
    if (t < S::NC) {
      const int cs = cell_case<N>(sf, n0, c);
      packed = s_ntri[cs] + ((cs != 0 && cs != 255) << 16);
      if (cdump) cdump[t] = (uint8_t)cs;
    }
    packed = (int)wave_sum_to63((uint32_t)packed);
    if ((t & 63) == 63) sred[t >> 6] = packed;
    __syncthreads();
    if (t == 0) {
      int sum = 0;
#pragma unroll
      for (int q = 0; q < TH / 64; ++q) sum += sred[q];
      cnt[(int64_t)s * n_elem + e] = sum & 0xffff;
      const int act = sum >> 16;
      if (active_total && act) atomicAdd((unsigned long long*)&active_total[s],
                                         (unsigned long long)act);
    }
    __syncthreads();
  }
}

// Emit triangles of every (isovalue, element) with a nonzero count.
template <int N, typename T>
__global__ void __launch_bounds__(Shape<N>::kCellThreads)
iso_emit(int64_t n_elem, const T* __restrict__ x, const T* __restrict__ y,
         const T* __restrict__ z, const T* __restrict__ field, int n_iso, IsoList<T> iso,
         const uint8_t* __restrict__ ntri_tab, const int8_t* __restrict__ tri_tab,
         const int32_t* __restrict__ cnt, const int64_t* __restrict__ offs, IsoOut<T> out,
         uint64_t* __restrict__ keys) {
  using S = Shape<N>;
  constexpr int TH = S::kCellThreads;
  constexpr int P = S::P;
  __shared__ T sf[S::NP], sx[S::NP], sy[S::NP], sz[S::NP];
  __shared__ uint8_t s_ntri[256];
  __shared__ int8_t s_tri[256 * kMcMaxTri * 3];
  __shared__ uint8_t s_case[S::NC];
  __shared__ uint16_t s_desc[S::NC * kMcMaxTri];
  __shared__ int32_t s_wave[TH / 64];
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
  for (int s = 0; s < n_iso; ++s) {
    const int64_t flat = (int64_t)s * n_elem + e;
    if (cnt[flat] == 0) continue;
    int64_t g = offs[flat];
    T* dst = out.ptr[0];
    int64_t cap = out.cap[0];
    if (out.per_iso) {
      g -= offs[(int64_t)s * n_elem];
      dst = out.ptr[s];
      cap = out.cap[s];
    }
    emit_element<N, TH>(iso.v[s], StridedNode<P, P * P>{}, StridedNode<P, P * P>{}, sf, sx, sy,
                        sz, s_ntri, s_tri,
                        s_case, s_desc, s_wave, dst, g, cap, out.per_iso ? nullptr : keys,
                        base);
  }
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan of int32 counts into int64 offsets
// ---------------------------------------------------------------------------

constexpr int kScanThreads = 256;

// Tile sums; a tile is kScanThreads x ITEMS counts (scan_tile).
template <int ITEMS>
__global__ void __launch_bounds__(kScanThreads)
scan_reduce(const int32_t* __restrict__ cnt, int64_t count, int64_t* __restrict__ partial) {
  __shared__ int64_t sred[kScanThreads / 64];
  const int64_t start = (int64_t)blockIdx.x * (kScanThreads * ITEMS);
  int64_t s = 0;
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
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

// Tiles' exclusive offsets.  FOLD: partial holds the tiles' sums, not yet
// scanned (nb <= kScanFold), and each workgroup adds up the sums of the
// tiles before it, which saves the one-workgroup scan of the partials.
constexpr int64_t kScanFold = 1024;
template <bool FOLD, int ITEMS>
__global__ void __launch_bounds__(kScanThreads)
scan_apply(const int32_t* __restrict__ cnt, int64_t count, const int64_t* __restrict__ partial,
           int64_t nb, int64_t* __restrict__ offs) {
  __shared__ int64_t sred[kScanThreads / 64];
  const int64_t start =
      (int64_t)blockIdx.x * (kScanThreads * ITEMS) + (int64_t)threadIdx.x * ITEMS;
  int32_t v[ITEMS];
  int64_t s = 0;
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    v[r] = (start + r < count) ? cnt[start + r] : 0;
    s += v[r];
  }
  int64_t base;
  if constexpr (FOLD) {
    int64_t b = 0;
    for (int64_t i = threadIdx.x; i < (int64_t)blockIdx.x; i += kScanThreads) b += partial[i];
    base = block_sum<kScanThreads>(b, sred);
  } else {
    base = partial[blockIdx.x];
  }
  int64_t total;
  int64_t run = base + block_exclusive_scan<kScanThreads>(s, sred, &total);
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    if (start + r < count) offs[start + r] = run;
    run += v[r];
  }
  if (blockIdx.x == nb - 1 && threadIdx.x == 0) offs[count] = FOLD ? base + total : partial[nb];
}

// Per-isovalue totals and the overflow flag, from the exclusive offsets
// (thread s < n_iso takes isovalue s).
template <typename T>
__device__ __forceinline__ void write_totals(int s, const int64_t* __restrict__ offs,
                                             int64_t n_elem, int n_iso,
                                             int64_t* __restrict__ tri_count,
                                             const IsoOut<T>& out, int32_t* __restrict__ status) {
  if (s < n_iso) {
    const int64_t c = offs[(int64_t)(s + 1) * n_elem] - offs[(int64_t)s * n_elem];
    tri_count[s] = c;
    if (status && out.per_iso && c > out.cap[s]) atomicOr(status, SEM_FLAG_TRI_OVERFLOW);
  }
  if (s == 0 && status && !out.per_iso && offs[(int64_t)n_iso * n_elem] > out.cap[0])
    atomicOr(status, SEM_FLAG_TRI_OVERFLOW);
}

template <typename T>
__global__ void iso_totals(const int64_t* __restrict__ offs, int64_t n_elem, int n_iso,
                           int64_t* __restrict__ tri_count, IsoOut<T> out,
                           int32_t* __restrict__ status) {
  write_totals<T>(threadIdx.x, offs, n_elem, n_iso, tri_count, out, status);
}

__global__ void fill_i64(int64_t* __restrict__ p, int n, int64_t value) {
  const int s = threadIdx.x;
  if (s < n) p[s] = value;
}

// ---------------------------------------------------------------------------
// N = 7, FP64 extraction: Q + triangle counts, scan, emission
// ---------------------------------------------------------------------------
//
// qcount_dma7 computes Q and |omega| from the six staged tiles, keeps Q in
// LDS and counts every isovalue's triangles and active cells per element.
// The counts then go through the device-wide exclusive scan, and emit_direct
// re-stages the Q and coordinate tiles of the elements that have triangles
// and writes them at their offsets.  (A single pass with a decoupled
// look-back saves that re-read, but on MI355X its chain of device-scope
// polls across the eight XCDs cost more than the re-read does.)
//
// qcount_dma7 runs four waves per element on the swizzled tile layout
// above, wave h (0..3) owning nodes i = h and 7 - h of r-line (j, k) =
// lane.  Waves 0, 1 differentiate the s-lines and waves 2, 3 the t-lines,
// half a line each, in the even-odd form of D.  With two nodes per lane
// (112 VGPRs) four waves fit on a SIMD to hide the load and LDS latencies.

// One 4 KiB tile with four waves: wave h issues chunk group h.
__device__ __forceinline__ void dma_tile4(const double* __restrict__ src, double* raw, int h,
                                          int lane) {
  const int s = 64 * h + lane;
  const int row = s >> 2, k = row >> 3, j = (row & 7) ^ (k & 1);
  const int ip = (s & 3) ^ ((j >> 1) & 3);
  lds_load16(src + 2 * (ip + 4 * j + 32 * k), raw + 128 * h);
}

// Even-odd form of an 8-point line derivative (D[7-i][7-m] = -D[i][m]):
// with e_m = g_m + g_{7-m}, o_m = g_m - g_{7-m} (m < 4),
// A[i][m] = (D[i][m] + D[i][7-m]) / 2 and B[i][m] = (D[i][m] - D[i][7-m]) / 2,
//   (D g)_i = R_i + P_i,  (D g)_{7-i} = R_i - P_i  (i < 4),
//   P_i = sum_m A[i][m] e_m,  R_i = sum_m B[i][m] o_m.
// Half the multiplies of the direct form, and a pair of outputs needs one
// row of A and B only.
__device__ __forceinline__ void eo_split(const double (&g)[8], double (&e)[4], double (&o)[4]) {
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    e[m] = g[m] + g[7 - m];
    o[m] = g[m] - g[7 - m];
  }
}
__device__ __forceinline__ void eo_pair(const double* __restrict__ eo, int i,
                                        const double (&e)[4], const double (&o)[4],
                                        double& lo, double& hi) {
  double P = coef(eo, 4 * i) * e[0], R = coef(eo, 16 + 4 * i) * o[0];
#pragma unroll
  for (int m = 1; m < 4; ++m) {
    P = fma(coef(eo, 4 * i + m), e[m], P);
    R = fma(coef(eo, 16 + 4 * i + m), o[m], R);
  }
  lo = R + P;
  hi = R - P;
}

// A lane's tile offsets in the swizzled layout, the same for every field:
// its r-line's four 16-byte chunks and the eight nodes of its s-line (waves
// 0, 1) or t-line (waves 2, 3).  Computed once per element and held in
// registers (the swizzle costs several instructions per offset).
struct Dma7Lane {
  int r[4];
  int g[8];
};
__device__ __forceinline__ Dma7Lane dma7_lane(int h, int p) {
  const int j = p & 7, k = p >> 3;
  Dma7Lane L;
#pragma unroll
  for (int ip = 0; ip < 4; ++ip) {
    L.r[ip] = 2 * dma7::slot(k, j, ip);
    asm volatile("" : "+v"(L.r[ip]));
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    L.g[m] = h < 2 ? dma7::at(j, m, k) : dma7::at(j, k, m);
    asm volatile("" : "+v"(L.g[m]));
  }
  return L;
}

// One field with four waves: wave h owns nodes i = h and 7 - h of r-line
// (j, k) = lane; waves 0, 1 differentiate s-lines, waves 2, 3 t-lines, each
// the output pairs (r, 7 - r) for r = 2(h&1) and 2(h&1) + 1.
__device__ __forceinline__ void dma_pass4(const double* __restrict__ raw,
                                          const double* __restrict__ eo, double* __restrict__ S,
                                          double* __restrict__ Tt, int h, int p,
                                          const Dma7Lane& L, double (&fr)[2], double (&fs)[2],
                                          double (&ft)[2]) {
  using Q = Pen<7>;
  const int j = p & 7, k = p >> 3;
  double f[8], e[4], o[4];
#pragma unroll
  for (int ip = 0; ip < 4; ++ip) {
    const double2 v = *reinterpret_cast<const double2*>(raw + L.r[ip]);
    f[2 * ip] = v.x;
    f[2 * ip + 1] = v.y;
  }
  eo_split(f, e, o);
  eo_pair(eo, h, e, o, fr[0], fr[1]);
  double g[8], out[4];
  const int r0 = 2 * (h & 1);
  // s-line at (i, k) = (j, k) of this lane's index (h < 2), else t-line at
  // (i, j) = (j, k)
#pragma unroll
  for (int m = 0; m < 8; ++m) g[m] = raw[L.g[m]];
  eo_split(g, e, o);
  eo_pair(eo, r0, e, o, out[0], out[1]);
  eo_pair(eo, r0 + 1, e, o, out[2], out[3]);
  const int idx[4] = {r0, 7 - r0, r0 + 1, 6 - r0};
  if (h < 2) {
#pragma unroll
    for (int q = 0; q < 4; ++q) S[Q::at(j, idx[q], k)] = out[q];
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) Tt[Q::at(j, k, idx[q])] = out[q];
  }
  lds_barrier();
  fs[0] = S[Q::at(h, j, k)];
  fs[1] = S[Q::at(7 - h, j, k)];
  ft[0] = Tt[Q::at(h, j, k)];
  ft[1] = Tt[Q::at(7 - h, j, k)];
  lds_barrier();
}

// Keep a value materialised here (the compiler may not defer its
// computation past later barriers, which would keep its inputs live).
__device__ __forceinline__ void pin(double& x) { asm volatile("" : "+v"(x)); }

// COUNT: also count every isovalue's triangles and active cells per element
// from the Q tile (sem_extract); otherwise Q, |omega| and the range only.
template <bool COUNT>
__device__ __forceinline__ void qcount_dma7_elem(
    int64_t e, int t, int64_t n_elem, const double* __restrict__ eo, const double* __restrict__ x,
    const double* __restrict__ y, const double* __restrict__ z, const double* __restrict__ u,
    const double* __restrict__ v, const double* __restrict__ w, double* __restrict__ q,
    double* __restrict__ om, double* __restrict__ qmm, int n_iso, const IsoList<double>& iso,
    const uint8_t* __restrict__ ntri_tab, int32_t* __restrict__ cnt,
    int64_t* __restrict__ active, int32_t* __restrict__ status) {
  __builtin_assume(t >= 0 && t < 256);
  __builtin_assume(e >= 0);
  constexpr int NC = 343;
  __shared__ double s_xyz[3][512];
  __shared__ double s_uvw[3][512];
  __shared__ double s_S[Pen<7>::SZ];
  __shared__ double s_T[Pen<7>::SZ];
  __shared__ double s_red[8];
  __shared__ uint32_t s_rows[32];
  const int h = __builtin_amdgcn_readfirstlane(t >> 6);
  const int p = t & 63;
  const int64_t base = e * 512;
  // the case-table entry is loaded first and stored once every load is in
  const uint8_t nt_own = COUNT ? ntri_tab[t] : 0;
  dma_tile4(x + base, s_xyz[0], h, p);
  dma_tile4(y + base, s_xyz[1], h, p);
  dma_tile4(z + base, s_xyz[2], h, p);
  dma_tile4(u + base, s_uvw[0], h, p);
  dma_tile4(v + base, s_uvw[1], h, p);
  dma_tile4(w + base, s_uvw[2], h, p);
  // coordinate tiles (the three velocity loads may stay in flight)
  __builtin_amdgcn_s_waitcnt(waitcnt_vm_lds(3));
  barrier_after_wait();
  double xr[2], xs[2], xt[2], yr[2], ys[2], yt[2], zr[2], zs[2], zt[2];
  const Dma7Lane lane_off = dma7_lane(h, p);
  dma_pass4(s_xyz[0], eo, s_S, s_T, h, p, lane_off, xr, xs, xt);
  dma_pass4(s_xyz[1], eo, s_S, s_T, h, p, lane_off, yr, ys, yt);
  dma_pass4(s_xyz[2], eo, s_S, s_T, h, p, lane_off, zr, zs, zt);
  // the chain rule runs on the adjugate of J (det J times J^-1); Q takes
  // the factor 1 / det^2 and |omega| the factor 1 / |det| once per node
  InvJac<double> kk[2];
  double inv[2];
  int bad = 0;
#pragma unroll
  for (int ii = 0; ii < 2; ++ii)
    bad |= !adjugate_jacobian(xr[ii], xs[ii], xt[ii], yr[ii], ys[ii], yt[ii], zr[ii], zs[ii],
                              zt[ii], kk[ii], inv[ii]);
#pragma unroll
  for (int ii = 0; ii < 2; ++ii) {
    pin(kk[ii].rx); pin(kk[ii].ry); pin(kk[ii].rz); pin(kk[ii].sx); pin(kk[ii].sy);
    pin(kk[ii].sz); pin(kk[ii].tx); pin(kk[ii].ty); pin(kk[ii].tz); pin(inv[ii]);
  }
  __builtin_amdgcn_s_waitcnt(waitcnt_vm_lds(0));
  barrier_after_wait();
  double fr[2], fs[2], ft[2], a01[2], a02[2], a12[2], qv[2], ov[2];
  dma_pass4(s_uvw[0], eo, s_S, s_T, h, p, lane_off, fr, fs, ft);
#pragma unroll
  for (int ii = 0; ii < 2; ++ii) {
    const InvJac<double>& K = kk[ii];
    const double a00 = fr[ii] * K.rx + fs[ii] * K.sx + ft[ii] * K.tx;
    a01[ii] = fr[ii] * K.ry + fs[ii] * K.sy + ft[ii] * K.ty;
    a02[ii] = fr[ii] * K.rz + fs[ii] * K.sz + ft[ii] * K.tz;
    qv[ii] = a00 * a00;
    pin(qv[ii]); pin(a01[ii]); pin(a02[ii]);
  }
  dma_pass4(s_uvw[1], eo, s_S, s_T, h, p, lane_off, fr, fs, ft);
#pragma unroll
  for (int ii = 0; ii < 2; ++ii) {
    const InvJac<double>& K = kk[ii];
    const double a10 = fr[ii] * K.rx + fs[ii] * K.sx + ft[ii] * K.tx;
    const double a11 = fr[ii] * K.ry + fs[ii] * K.sy + ft[ii] * K.ty;
    a12[ii] = fr[ii] * K.rz + fs[ii] * K.sz + ft[ii] * K.tz;
    qv[ii] = qv[ii] + a11 * a11 + 2.0 * (a01[ii] * a10);
    const double w3 = a10 - a01[ii];
    ov[ii] = w3 * w3;
    pin(qv[ii]); pin(ov[ii]); pin(a12[ii]);
  }
  dma_pass4(s_uvw[2], eo, s_S, s_T, h, p, lane_off, fr, fs, ft);
#pragma unroll
  for (int ii = 0; ii < 2; ++ii) {
    const InvJac<double>& K = kk[ii];
    const double a20 = fr[ii] * K.rx + fs[ii] * K.sx + ft[ii] * K.tx;
    const double a21 = fr[ii] * K.ry + fs[ii] * K.sy + ft[ii] * K.ty;
    const double a22 = fr[ii] * K.rz + fs[ii] * K.sz + ft[ii] * K.tz;
    qv[ii] = -0.5 * (qv[ii] + a22 * a22 + 2.0 * (a02[ii] * a20 + a12[ii] * a21)) *
             (inv[ii] * inv[ii]);
    const double w1 = a21 - a12[ii], w2 = a02[ii] - a20;
    ov[ii] = sqrt_refined(ov[ii] + w1 * w1 + w2 * w2) * fabs(inv[ii]);
  }
  const int j = p & 7, k = p >> 3;
  // Q and |omega| go out through LDS tiles (free after the u and v passes):
  // each lane then stores 16 contiguous bytes, a wave 1 KiB
  double* QT = s_uvw[0];
  double* OT = s_uvw[1];
  double mn = pos_inf<double>(), mx = neg_inf<double>();
#pragma unroll
  for (int ii = 0; ii < 2; ++ii) {
    QT[dma7::at(ii ? 7 - h : h, j, k)] = qv[ii];
    OT[dma7::at(ii ? 7 - h : h, j, k)] = ov[ii];
    const double c = qv[ii] != qv[ii] ? neg_inf<double>() : qv[ii];
    mn = c < mn ? c : mn;
    mx = c > mx ? c : mx;
  }
  wave_minmax(mn, mx);
  if (p == 63) {
    s_red[h] = mn;
    s_red[4 + h] = mx;
  }
  // Counting works on isovalues four at a time: a node's word holds bit
  // (Q > c_s) at bit 8s, so the eight corner words of a cell, each shifted
  // by its vertex number and summed, give the four cell cases as bytes. The
  // derivative tiles are free now: S holds the node words, T the case table
  // as triangles + (1 << 8) per non-trivial case.
  uint32_t* s_bits = reinterpret_cast<uint32_t*>(s_S);
  int32_t* s_tab = reinterpret_cast<int32_t*>(s_T);
  const int node0 = h + 8 * j + 64 * k, node1 = 7 - h + 8 * j + 64 * k;
  if constexpr (COUNT) {
    s_tab[t] = case_count_entry8(t, nt_own);
    s_bits[node0] = iso_bits4(qv[0], iso, 0, n_iso);
    s_bits[node1] = iso_bits4(qv[1], iso, 0, n_iso);
  }
  // an inverted element (rare) is flagged by its own lanes: no block vote
  if (bad && status) atomicOr(status, SEM_FLAG_BAD_JACOBIAN);
  __syncthreads();               // publishes the tiles, s_red and the node words
  {
    // node pair (2t, 2t + 1) of the natural layout sits in one 16-byte slot
    const int n = 2 * t;
    const int sl = 2 * dma7::slot(n >> 6, (n >> 3) & 7, (n & 7) >> 1);
    if (q) *reinterpret_cast<double2*>(q + base + n) = *reinterpret_cast<const double2*>(QT + sl);
    if (om)
      *reinterpret_cast<double2*>(om + base + n) = *reinterpret_cast<const double2*>(OT + sl);
  }
  mn = fmin(fmin(s_red[0], s_red[1]), fmin(s_red[2], s_red[3]));
  mx = fmax(fmax(s_red[4], s_red[5]), fmax(s_red[6], s_red[7]));
  if (qmm && t == 0) {
    qmm[2 * e] = mn;
    qmm[2 * e + 1] = mx;
  }
  if constexpr (COUNT) {
    // cell t, and cell t + 256 for the threads t < 87 (waves 0 and 1 only);
    // corner 0 of a cell at its natural node index, the others at fixed
    // offsets from it
    constexpr int NC2 = NC - 256;
    const bool two = t < NC2;
    const int c1 = two ? t + 256 : t;
    const int cb[2] = {cell_base7(t), cell_base7(c1)};
    for (int g = 0; g < n_iso; g += 4) {
      const int m = n_iso - g < 4 ? n_iso - g : 4;
      if (g > 0) {   // every read of the previous words is behind the last barrier
        s_bits[node0] = iso_bits4(qv[0], iso, g, n_iso);
        s_bits[node1] = iso_bits4(qv[1], iso, g, n_iso);
        __syncthreads();
      }
      // an element outside every isovalue's range of the group has only
      // trivial cases (NaN nodes count as below; mn is -inf then)
      bool live = false;
      for (int s = 0; s < m; ++s) live |= (mx > iso.v[g + s]) && !(mn > iso.v[g + s]);
      // a lane's cells: per isovalue s, triangles + (active << 8) in the
      // 16-bit half s & 1 of word s >> 1 (publish_rows)
      uint32_t pw[2] = {0u, 0u};
      if (live) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          if (r == 1 && h >= 2) break;
          uint32_t word = 0;
#pragma unroll
          for (int vtx = 0; vtx < 8; ++vtx)
            word += s_bits[cb[r] + (vtx & 1) + 8 * ((vtx >> 1) & 1) + 64 * (vtx >> 2)] << vtx;
          if (r == 0 || two) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
              if (s < m) pw[s >> 1] += (uint32_t)s_tab[(word >> (8 * s)) & 255] << (16 * (s & 1));
          }
        }
      }
      publish_rows<4>(pw, m, g, t, s_rows, cnt, n_elem, e, active);
    }
  }
}

template <bool COUNT>
__global__ void __launch_bounds__(256)
qcount_dma7(int64_t n_elem, const double* __restrict__ eo, const double* __restrict__ x,
             const double* __restrict__ y, const double* __restrict__ z,
             const double* __restrict__ u, const double* __restrict__ v,
             const double* __restrict__ w, double* __restrict__ q, double* __restrict__ om,
             double* __restrict__ qmm, int n_iso, IsoList<double> iso,
             const uint8_t* __restrict__ ntri_tab, int32_t* __restrict__ cnt,
             int64_t* __restrict__ active, int32_t* __restrict__ status) {
  qcount_dma7_elem<COUNT>(blockIdx.x, threadIdx.x, n_elem, eo, x, y, z, u, v, w, q, om, qmm,
                          n_iso, iso, ntri_tab, cnt, active, status);
}

// Emission for N = 7, FP64: elements with triangles stage their field and
// coordinate tiles with direct loads and emit through emit_element.

// Odd N (an even number of nodes per edge: every tile is a whole number of
// 16-byte chunks and starts 16-byte aligned): a tile arrives in natural
// node order, wave h issuing the 1 KiB instructions h, h + 2, ... (lanes
// past the tile's end load nothing).
template <int N, typename T>
__device__ __forceinline__ void dma_tile_natural(const T* __restrict__ src, T* raw, int h,
                                                 int lane) {
  constexpr int CH = (N + 1) * (N + 1) * (N + 1) * (int)sizeof(T) / 16;   // 16-byte chunks
  static_assert((N + 1) * (N + 1) * (N + 1) * sizeof(T) % 16 == 0, "whole chunks");
#pragma unroll
  for (int q = h; q * 64 < CH; q += 2) {
    if (q * 64 + lane < CH)
      lds_load16(reinterpret_cast<const double*>(src) + 2 * (q * 64 + lane),
                 reinterpret_cast<double*>(raw) + 128 * q);
  }
}

// emit_direct<N, T>: the element's tiles and the case tables by direct loads,
// two waves per element (odd N; N = 7 FP64 uses the swizzled tile).
// Element tile of any order into LDS for two waves: direct loads where the
// tile is a whole number of 16-byte chunks at a 16-byte aligned address
// (odd N), plain loads otherwise.  Consumers wait with
// s_waitcnt(vm, lgkm = 0) and a barrier.
template <int N, typename T>
__device__ __forceinline__ void tile2_lds(const T* __restrict__ src, T* dst, int h, int lane) {
  constexpr int NP = (N + 1) * (N + 1) * (N + 1);
  if constexpr (N % 2 == 1) {
    dma_tile_natural<N>(src, dst, h, lane);
  } else {
    for (int q = 64 * h + lane; q < NP; q += 128) dst[q] = src[q];
  }
}

// Emission of element e (two waves): every isovalue with a nonzero count
// writes its triangles at offs[s * n_elem + e] of out (or of out.ptr[s],
// relative to the isovalue's first offset, when out.per_iso).
template <int N, typename T, class IL = IsoList<T>, class OUT = IsoOut<T>>
__device__ __forceinline__ void emit_elem(int64_t e, int t, int64_t n_elem,
                                          const T* __restrict__ x, const T* __restrict__ y,
                                          const T* __restrict__ z, const T* __restrict__ field,
                                          int n_iso, const IL& iso, const OUT& out,
                                          const uint8_t* __restrict__ ntri_tab,
                                          const int32_t* __restrict__ cnt,
                                          const int64_t* __restrict__ offs,
                                          uint64_t* __restrict__ keys) {
  constexpr int P = N + 1, NP = P * P * P, NC = N * N * N;
  constexpr bool SWZ = N == 7 && std::is_same<T, double>::value;
  // The coordinate tiles are staged in LDS too, except for FP32 at N = 9,
  // which reads the coordinates where the vertices need them (edge
  // endpoints only, through the caches) and so needs 16 instead of 28 KB of
  // LDS. Measured: staged is faster for FP64 N = 7 (0.319 against 0.379 ms)
  // and FP32 N = 7 (the FP32 step 0.679 against 0.712 ms); reading made the
  // FP32 batched step (orders 5, 7, 9) 11.90 instead of 12.20 ms.
  constexpr bool XYZ = std::is_same<T, double>::value || N <= 7;
  __shared__ __attribute__((aligned(16))) T s_f[NP];
  __shared__ __attribute__((aligned(16))) T s_x[XYZ ? NP : 1];
  __shared__ __attribute__((aligned(16))) T s_y[XYZ ? NP : 1];
  __shared__ __attribute__((aligned(16))) T s_z[XYZ ? NP : 1];
  static_assert(256 + 256 * kMcMaxTri * 3 == 4096, "tables fill one 4 KiB block");
  __shared__ uint4 s_tab[16];      // triangle counts (256 B)
  __shared__ uint8_t s_case[NC];
  __shared__ uint16_t s_desc[NC * kMcMaxTri];
  __shared__ int32_t s_wave[2];
  const uint8_t* s_ntri = reinterpret_cast<const uint8_t*>(s_tab);
  const int8_t* s_tri = reinterpret_cast<const int8_t*>(ntri_tab) + 256;   // through the caches
  __builtin_assume(t >= 0 && t < 128);
  const int h = __builtin_amdgcn_readfirstlane(t >> 6);
  const int p = t & 63;
  bool any = false;
  for (int s = 0; s < n_iso; ++s) any = any || cnt[(int64_t)s * n_elem + e] > 0;
  if (!any) return;
  const int64_t base = e * NP;
  // the triangle counts (256 B) and the tiles arrive by direct loads before
  // the one wait below; the case table (3.75 KiB) is read through the caches
  // in the vertex loop, which takes the FP64 workgroup from 24.3 to 20.4 KB
  // of LDS, six to eight per CU (emission 0.319 -> 0.307 ms on the channel
  // snapshot)
  if (h == 0 && p < 16)
    lds_load16(reinterpret_cast<const double*>(ntri_tab) + 2 * p,
               reinterpret_cast<double*>(s_tab));
  if constexpr (SWZ) {
    dma_tile(field + base, s_f, h, p);
    dma_tile(x + base, s_x, h, p);
    dma_tile(y + base, s_y, h, p);
    dma_tile(z + base, s_z, h, p);
  } else {
    tile2_lds<N>(field + base, s_f, h, p);
    if constexpr (XYZ) {
      tile2_lds<N>(x + base, s_x, h, p);
      tile2_lds<N>(y + base, s_y, h, p);
      tile2_lds<N>(z + base, s_z, h, p);
    }
  }
  const T* gx = XYZ ? s_x : x + base;
  const T* gy = XYZ ? s_y : y + base;
  const T* gz = XYZ ? s_z : z + base;
  __builtin_amdgcn_s_waitcnt(waitcnt_vm_lds(0));
  barrier_after_wait();
  for (int s = 0; s < n_iso; ++s) {
    const int64_t flat = (int64_t)s * n_elem + e;
    if (cnt[flat] == 0) continue;
    int64_t g = offs[flat];
    T* dst = out.ptr[0];
    int64_t cap = out.cap[0];
    if (out.per_iso) {
      g -= offs[(int64_t)s * n_elem];
      dst = out.ptr[s];
      cap = out.cap[s];
    }
    if constexpr (SWZ)
      emit_element<7, 128>(iso.v[s], DmaNode{}, DmaNode{}, s_f, gx, gy, gz, s_ntri, s_tri,
                           s_case, s_desc, s_wave, dst, g, cap, out.per_iso ? nullptr : keys,
                           base);
    else
      emit_element<N, 128>(iso.v[s], StridedNode<P, P * P>{}, StridedNode<P, P * P>{}, s_f,
                           gx, gy, gz, s_ntri, s_tri, s_case, s_desc, s_wave, dst, g, cap,
                           out.per_iso ? nullptr : keys, base);
  }
}

template <int N, typename T>
__global__ void __launch_bounds__(128)
emit_direct(int64_t n_elem, const T* __restrict__ x, const T* __restrict__ y,
            const T* __restrict__ z, const T* __restrict__ field, int n_iso,
            IsoList<T> iso, IsoOut<T> out, const uint8_t* __restrict__ ntri_tab,
            const int32_t* __restrict__ cnt, const int64_t* __restrict__ offs,
            uint64_t* __restrict__ keys, int64_t* __restrict__ tri_count,
            int32_t* __restrict__ status) {
  // the last workgroup also writes the totals (in place of a kernel of its own)
  if (blockIdx.x == gridDim.x - 1)
    write_totals<T>(threadIdx.x, offs, n_elem, n_iso, tri_count, out, status);
  emit_elem<N, T>(blockIdx.x, threadIdx.x, n_elem, x, y, z, field, n_iso, iso, out, ntri_tab,
                  cnt, offs, keys);
}

// count_direct<N, T>: the count pass of the two-pass isosurface for odd N:
// the field tile (and the triangle-count table) by direct loads, two waves
// per element, one packed block sum (triangles | active cells << 16) per
// isovalue; elements the range excludes write zero counts without loading.
template <int N, typename T, class IL = IsoList<T>>
__device__ __forceinline__ void count_elem(int64_t e, int t, int64_t n_elem,
                                           const T* __restrict__ field, const T* __restrict__ mm,
                                           int n_iso, const IL& iso,
                                           const uint8_t* __restrict__ ntri_tab,
                                           int32_t* __restrict__ cnt,
                                           int64_t* __restrict__ active_total,
                                           uint8_t* __restrict__ case_idx) {
  constexpr int P = N + 1, NP = P * P * P, NC = N * N * N, R = (NC + 127) / 128;
  __shared__ __attribute__((aligned(16))) T sf[NP];
  __shared__ __attribute__((aligned(16))) uint8_t s_ntri[256];
  __shared__ T red[4];
  __shared__ int32_t s_sum[2];
  __builtin_assume(t >= 0 && t < 128);
  const int h = __builtin_amdgcn_readfirstlane(t >> 6);
  const int lane = t & 63;
  T mn = pos_inf<T>(), mx = neg_inf<T>();
  bool need = true;
  if (mm) {
    mn = mm[2 * e];
    mx = mm[2 * e + 1];
    need = false;
    for (int s = 0; s < n_iso; ++s) need = need || ((mx > iso.v[s]) && !(mn > iso.v[s]));
  }
  if (!need) {
    // no isovalue inside the element's range: zero counts, uniform cases
    for (int s = 0; s < n_iso; ++s) {
      if (t == 0) cnt[(int64_t)s * n_elem + e] = 0;
      if (case_idx) {
        uint8_t* cd = case_idx + ((int64_t)s * n_elem + e) * NC;
        const uint8_t v = (mx > iso.v[s]) ? 255 : 0;
        for (int q = t; q < NC; q += 128) cd[q] = v;
      }
    }
    return;
  }
  if (h == 0 && lane < 16)
    lds_load16(reinterpret_cast<const double*>(ntri_tab) + 2 * lane,
               reinterpret_cast<double*>(s_ntri));
  tile2_lds<N>(field + e * NP, sf, h, lane);
  __builtin_amdgcn_s_waitcnt(waitcnt_vm_lds(0));
  barrier_after_wait();
  if (!mm) {
    T a = pos_inf<T>(), b = neg_inf<T>();
    for (int q = t; q < NP; q += 128) {
      T val = sf[q];
      if (val != val) val = neg_inf<T>();
      a = val < a ? val : a;
      b = val > b ? val : b;
    }
    block_minmax<T, 128>(a, b, red);
    mn = a;
    mx = b;
  }
  // corners of this thread's cells, loaded once
  T cv[R][8];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int cc = t + 128 * r < NC ? t + 128 * r : 0;
    const int n0 = cc % N + P * ((cc / N) % N) + P * P * (cc / (N * N));
#pragma unroll
    for (int vtx = 0; vtx < 8; ++vtx)
      cv[r][vtx] = sf[n0 + (vtx & 1) + P * ((vtx >> 1) & 1) + P * P * (vtx >> 2)];
  }
  for (int s = 0; s < n_iso; ++s) {
    const T c = iso.v[s];
    const bool straddle = (mx > c) && !(mn > c);
    uint8_t* cd = case_idx ? case_idx + ((int64_t)s * n_elem + e) * NC : nullptr;
    int packed = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int cell = t + 128 * r;
      if (cell >= NC) continue;
      int cs = 0;
      if (straddle) {
#pragma unroll
        for (int vtx = 7; vtx >= 0; --vtx) cs = cs + cs + (cv[r][vtx] > c);
        packed += s_ntri[cs] + ((cs != 0 && cs != 255) << 16);
      } else {
        cs = (mx > c) ? 255 : 0;
      }
      if (cd) cd[cell] = (uint8_t)cs;
    }
    if (!straddle) {
      if (t == 0) cnt[(int64_t)s * n_elem + e] = 0;
      continue;
    }
    packed = (int)wave_sum_to63((uint32_t)packed);
    if (lane == 63) s_sum[h] = packed;
    __syncthreads();
    if (t == 0) {
      const int sum = s_sum[0] + s_sum[1];
      cnt[(int64_t)s * n_elem + e] = sum & 0xffff;
      const int act = sum >> 16;
      if (active_total && act)
        atomicAdd((unsigned long long*)&active_total[s], (unsigned long long)act);
    }
    __syncthreads();
  }
}

template <int N, typename T>
__global__ void __launch_bounds__(128)
count_direct(int64_t n_elem, const T* __restrict__ field, const T* __restrict__ mm,
             int n_iso, IsoList<T> iso, const uint8_t* __restrict__ ntri_tab,
             int32_t* __restrict__ cnt, int64_t* __restrict__ active_total,
             uint8_t* __restrict__ case_idx) {
  count_elem<N, T>(blockIdx.x, threadIdx.x, n_elem, field, mm, n_iso, iso, ntri_tab, cnt,
                   active_total, case_idx);
}

// ---------------------------------------------------------------------------
// mixed precision, N = 7, FP32 storage: derivative contractions on MFMA
// ---------------------------------------------------------------------------
//
// The 1-D contractions run as v_mfma_f32_16x16x32_{bf16,f16}: low-precision
// operands, FP32 accumulation.  One workgroup of four waves per element; for
// each field and direction wave w differentiates the 16 lines 16w..16w+15:
//   rows     i = output node along the line (rows 8..15 are zero),
//   columns  the 16 lines,
//   depth    the 8 line values spread over the four lane groups (group g
//            holds values m0 = 2g and m1 = 2g + 1), each with the products
//            the mode needs:
//   plain            D_hi (f - f_0)_hi
//   split (x3)       D_hi f_hi + D_lo f_hi + D_hi f_lo   (Henry, Tang &
//                    Heinecke 2019: the lo*lo term is dropped)
// where x_hi = round(x) to the operand format and x_lo = round(x - x_hi).
// In the FP16 split the lo parts are scaled by 2^11 (out of FP16's subnormal
// range; Ootomo & Yokota 2022) and accumulate separately, then scaled back.
// Values enter line-shifted (f_m - f_0), which keeps the coordinates'
// absolute offset out of the rounding.  The Jacobian is inverted in FP64;
// the chain rule, Q and |omega| are FP32.

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

enum MixMode { kMixBF16 = 0, kMixFP16 = 1, kMixBF16x3 = 2, kMixFP16x3 = 3 };

template <int M>
struct MixT {
  typedef __bf16 E;
  typedef bf16x8 V;
};
template <>
struct MixT<kMixFP16> {
  typedef _Float16 E;
  typedef f16x8 V;
};
template <>
struct MixT<kMixFP16x3> {
  typedef _Float16 E;
  typedef f16x8 V;
};

constexpr float kF16LoScale = 2048.0f;   // 2^11

template <int M>
__device__ __forceinline__ f32x4 mfma_line(typename MixT<M>::V a, typename MixT<M>::V b) {
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  if constexpr (M == kMixBF16 || M == kMixBF16x3)
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, zero, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, zero, 0, 0, 0);
}

// A operands of one lane (row i = lane % 16, lane group g = lane / 16).
template <int M>
struct MixOps {
  typename MixT<M>::V a;    // main product
  typename MixT<M>::V ac;   // scaled correction (FP16 split only)
};

template <int M>
__device__ __forceinline__ MixOps<M> mix_ops(const double* __restrict__ d, int lane) {
  using E = typename MixT<M>::E;
  MixOps<M> o;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    o.a[q] = E(0.f);
    o.ac[q] = E(0.f);
  }
  const int i = lane & 15, g = lane >> 4;
  // rows 8..15 are zero: their values are selected to zero after an
  // unconditional load (row i & 7), so that no branch holds the caller's
  // later loads behind this load's wait
  const double r0 = d[(i & 7) * 8 + 2 * g], r1 = d[(i & 7) * 8 + 2 * g + 1];
  const double d0 = i < 8 ? r0 : 0.0, d1 = i < 8 ? r1 : 0.0;
  const E h0 = E((float)d0), h1 = E((float)d1);
  if constexpr (M == kMixBF16x3) {
    const E l0 = E((float)(d0 - (double)(float)h0));
    const E l1 = E((float)(d1 - (double)(float)h1));
    o.a[0] = h0; o.a[1] = l0; o.a[2] = h0;
    o.a[3] = h1; o.a[4] = l1; o.a[5] = h1;
  } else {
    o.a[0] = h0;
    o.a[1] = h1;
    if constexpr (M == kMixFP16x3) {
      o.ac[0] = E((float)((d0 - (double)(float)h0) * kF16LoScale));
      o.ac[1] = h0;
      o.ac[2] = E((float)((d1 - (double)(float)h1) * kF16LoScale));
      o.ac[3] = h1;
    }
  }
  return o;
}

// Derivatives along one line set: v0, v1 are this lane's shifted values
// f[m0] - f[0], f[m1] - f[0]; lanes 0..31 receive the outputs of rows
// 4 (lane / 16) .. + 3 for line lane % 16.
template <int M>
__device__ __forceinline__ f32x4 mix_contract(const MixOps<M>& o, float v0, float v1) {
  using E = typename MixT<M>::E;
  typename MixT<M>::V b;
#pragma unroll
  for (int q = 0; q < 8; ++q) b[q] = E(0.f);
  const E h0 = E(v0), h1 = E(v1);
  if constexpr (M == kMixBF16x3) {
    const E l0 = E(v0 - (float)h0), l1 = E(v1 - (float)h1);
    b[0] = h0; b[1] = h0; b[2] = l0;
    b[3] = h1; b[4] = h1; b[5] = l1;
    return mfma_line<M>(o.a, b);
  } else {
    b[0] = h0;
    b[1] = h1;
    f32x4 acc = mfma_line<M>(o.a, b);
    if constexpr (M == kMixFP16x3) {
      typename MixT<M>::V bc;
#pragma unroll
      for (int q = 0; q < 8; ++q) bc[q] = E(0.f);
      bc[0] = h0;
      bc[1] = E((v0 - (float)h0) * kF16LoScale);
      bc[2] = h1;
      bc[3] = E((v1 - (float)h1) * kF16LoScale);
      const f32x4 c = mfma_line<M>(o.ac, bc);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = fmaf(c[r], 1.0f / kF16LoScale, acc[r]);
    }
    return acc;
  }
}

constexpr int kMixLS = 9;            // derivative tile: line stride (floats)
constexpr int kMixDT = 64 * kMixLS;  // one derivative tile

// One field (tile `f`, natural layout i + 8j + 64k) -> its three derivative
// tiles `dt` (line-major: dt[d * kMixDT + line * kMixLS + node along line]).
template <int M>
__device__ __forceinline__ void mix_field(const float* __restrict__ f, float* __restrict__ dt,
                                          const MixOps<M>& o, int wv, int lane) {
  const int n = lane & 15, g = lane >> 4;
  const int L = 16 * wv + n;
  const int lo = L & 7, hi = L >> 3;
  // line base and stride of direction r, s, t
  const int base[3] = {8 * L, lo + 64 * hi, L};
  const int stride[3] = {1, 8, 64};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float* line = f + base[d];
    const float f0 = line[0];
    const float v0 = line[(2 * g) * stride[d]] - f0;
    const float v1 = line[(2 * g + 1) * stride[d]] - f0;
    const f32x4 acc = mix_contract<M>(o, v0, v1);
    if (lane < 32) {
      float* out = dt + d * kMixDT + L * kMixLS + 4 * g;
#pragma unroll
      for (int r = 0; r < 4; ++r) out[r] = acc[r];
    }
  }
}

// (f_r, f_s, f_t) of node (i, j, k) from its field's derivative tiles.
__device__ __forceinline__ void mix_read(const float* __restrict__ dt, int i, int j, int k,
                                         float& fr, float& fs, float& ft) {
  fr = dt[(j + 8 * k) * kMixLS + i];
  fs = dt[kMixDT + (i + 8 * k) * kMixLS + j];
  ft = dt[2 * kMixDT + (i + 8 * j) * kMixLS + k];
}

// QC: Q, |omega| and the element range of Q from (x, y, z, u, v, w);
// otherwise the physical gradient of f = u into (o0, o1, o2).
// COUNT (with QC): also the per-(isovalue, element) triangle and active-cell
// counts from the element's Q tile.
template <int M, bool QC, bool COUNT = false>
__global__ void __launch_bounds__(256)
mixed7(const double* __restrict__ dmat, const float* __restrict__ x,
       const float* __restrict__ y, const float* __restrict__ z, const float* __restrict__ u,
       const float* __restrict__ v, const float* __restrict__ w, float* __restrict__ o0,
       float* __restrict__ o1, float* __restrict__ o2, float* __restrict__ qmm,
       int32_t* __restrict__ status, CountSink<float> sink) {
  static_assert(QC || !COUNT, "counting needs Q");
  constexpr int NF = QC ? 6 : 4;
  __shared__ float s_in[NF][512];
  __shared__ float s_d[2][3 * kMixDT];
  __shared__ float s_red[8];
  __shared__ int32_t s_tab[COUNT ? 256 : 1];
  __shared__ uint32_t s_rows[COUNT ? 32 : 1];
  const int t = threadIdx.x, lane = t & 63;
  __builtin_assume(t >= 0 && t < 256);
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int64_t base = (int64_t)blockIdx.x * 512;
  // the first 128 threads stage the 16-byte chunks of x, z, v, the others
  // those of y, u, w; every load is requested before the first LDS write (a
  // field picked by an index into a pointer list became a compare-and-select
  // chain that serialised the loads)
  const MixOps<M> ops = mix_ops<M>(dmat, lane);   // its loads first: in flight with the tiles'
  const bool hi = t >= 128;
  const int64_t off = base + 4 * (t & 127);
  const int slot = 4 * (t & 127);
  const float4 c0 = *reinterpret_cast<const float4*>((hi ? y : x) + off);
  const float4 c1 = *reinterpret_cast<const float4*>((hi ? u : z) + off);
  float4 c2 = make_float4(0.f, 0.f, 0.f, 0.f);
  if constexpr (NF == 6) c2 = *reinterpret_cast<const float4*>((hi ? w : v) + off);
  uint8_t nt_own = 0;
  if constexpr (COUNT) nt_own = sink.ntri[t];
  *reinterpret_cast<float4*>((hi ? s_in[1] : s_in[0]) + slot) = c0;
  *reinterpret_cast<float4*>((hi ? s_in[3] : s_in[2]) + slot) = c1;
  if constexpr (NF == 6) *reinterpret_cast<float4*>((hi ? s_in[5] : s_in[4]) + slot) = c2;
  if constexpr (COUNT) s_tab[t] = case_count_entry8(t, nt_own);
  __syncthreads();

  // owners: nodes t and t + 256
  int ni[2], nj[2], nk[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int nd = t + 256 * h;
    ni[h] = nd & 7;
    nj[h] = (nd >> 3) & 7;
    nk[h] = nd >> 6;
  }
  float gd[3][2][3];   // geometry: [coordinate][node][r, s, t]
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float* dt = s_d[c & 1];
    mix_field<M>(s_in[c], dt, ops, wv, lane);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) mix_read(dt, ni[h], nj[h], nk[h], gd[c][h][0], gd[c][h][1],
                                         gd[c][h][2]);
  }
  int bad = 0;
  InvJac<float> kk[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    InvJac<double> k64;
    bad |= !invert_jacobian<double>(gd[0][h][0], gd[0][h][1], gd[0][h][2], gd[1][h][0],
                                    gd[1][h][1], gd[1][h][2], gd[2][h][0], gd[2][h][1],
                                    gd[2][h][2], k64);
    kk[h] = InvJac<float>{(float)k64.rx, (float)k64.ry, (float)k64.rz,
                          (float)k64.sx, (float)k64.sy, (float)k64.sz,
                          (float)k64.tx, (float)k64.ty, (float)k64.tz};
  }
  float a[2][3][3];
#pragma unroll
  for (int c = 0; c < NF - 3; ++c) {
    float* dt = s_d[(3 + c) & 1];
    mix_field<M>(s_in[3 + c], dt, ops, wv, lane);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float fr, fs, ft;
      mix_read(dt, ni[h], nj[h], nk[h], fr, fs, ft);
      const InvJac<float>& K = kk[h];
      a[h][c][0] = fr * K.rx + fs * K.sx + ft * K.tx;
      a[h][c][1] = fr * K.ry + fs * K.sy + ft * K.ty;
      a[h][c][2] = fr * K.rz + fs * K.sz + ft * K.tz;
    }
  }
  // an inverted element (rare) is flagged by its own lanes: no block vote
  if (bad && status) atomicOr(status, SEM_FLAG_BAD_JACOBIAN);
  __syncthreads();
  if constexpr (!QC) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t o = base + t + 256 * h;
      o0[o] = a[h][0][0];
      o1[o] = a[h][0][1];
      o2[o] = a[h][0][2];
    }
  } else {
    float mn = pos_inf<float>(), mx = neg_inf<float>();
    float qn[2];
    uint32_t* bits = reinterpret_cast<uint32_t*>(s_in[0]);   // x was read in the first pass only
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float(&A)[3][3] = a[h];
      const float tr2 = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2] +
                        2.f * (A[0][1] * A[1][0] + A[0][2] * A[2][0] + A[1][2] * A[2][1]);
      const float w1 = A[2][1] - A[1][2], w2 = A[0][2] - A[2][0], w3 = A[1][0] - A[0][1];
      const float qv = -0.5f * tr2;
      const int64_t o = base + t + 256 * h;
      if (o0) o0[o] = qv;
      if (o1) o1[o] = vort_root(w1 * w1 + w2 * w2 + w3 * w3);
      qn[h] = qv;
      if constexpr (COUNT) bits[t + 256 * h] = iso_bits4<float>(qv, sink.iso, 0, sink.n_iso);
      const float c = qv != qv ? neg_inf<float>() : qv;
      mn = c < mn ? c : mn;
      mx = c > mx ? c : mx;
    }
    if (qmm || COUNT) {
      block_minmax<float, 256>(mn, mx, s_red);   // its barriers publish the Q tile
      if (qmm && t == 0) {
        qmm[2 * (int64_t)blockIdx.x] = mn;
        qmm[2 * (int64_t)blockIdx.x + 1] = mx;
      }
    }
    if constexpr (COUNT) {
      // cells t and t + 256 (t < 87); node words in natural order
      constexpr int NC = 343;
      int n0[2];
#pragma unroll
      for (int r = 0; r < 2; ++r) n0[r] = cell_base7(t + 256 * r < NC ? t + 256 * r : t);
      const int64_t e = blockIdx.x;
      const int n_iso = sink.n_iso;
      for (int g = 0; g < n_iso; g += 4) {
        const int m = n_iso - g < 4 ? n_iso - g : 4;
        if (g > 0) {   // every read of the previous words is behind the last barrier
#pragma unroll
          for (int h = 0; h < 2; ++h) bits[t + 256 * h] = iso_bits4<float>(qn[h], sink.iso, g, n_iso);
          __syncthreads();
        }
        bool live = false;   // (NaN nodes count as below; mn is -inf then)
        for (int s = 0; s < m; ++s) live |= (mx > sink.iso.v[g + s]) && !(mn > sink.iso.v[g + s]);
        uint32_t pw[2] = {0u, 0u};
        if (live) {
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            if (t + 256 * r >= NC) continue;
            const uint32_t word = cell_word<8, 64>(bits, n0[r]);
#pragma unroll
            for (int s = 0; s < 4; ++s)
              if (s < m) pw[s >> 1] += (uint32_t)s_tab[(word >> (8 * s)) & 255] << (16 * (s & 1));
          }
        }
        publish_rows<4>(pw, m, g, t, s_rows, sink.cnt, sink.n_elem, e, sink.active);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// batched snapshots: one persistent launch over every snapshot's elements
// ---------------------------------------------------------------------------
//
// Work item = `chunk` consecutive elements of one snapshot; snapshots may
// differ in order N and element count.  Each workgroup takes items
// blockIdx.x, blockIdx.x + gridDim.x, ... ; for an item it finds the
// snapshot (binary search over the items' prefix), stages the chunk's six
// tiles and D in LDS and computes Q, |omega| and the element ranges with
// the order's instantiation.  The chunk per (order, precision) is what the
// autotuner measured fastest: small elements leave threads idle unless
// several share a workgroup.

constexpr int kBatchThreads = 256;
constexpr int kBatchTile = 6144;   // LDS values for 6 fields x chunk x (N+1)^3

template <int N, typename T>
__device__ __forceinline__ int batch_chunk(const coef_t<N, T>* dmat, const T* const (&fp)[6], T* oq,
                                           T* oom, T* oqmm, int64_t e0, int ne, T* tiles,
                                           coef_t<N, T>* sd) {
  constexpr int P = N + 1, P3 = P * P * P;
  constexpr int MAXQ = kBatchTile / 6 / kBatchThreads;   // node values per thread
  const int t = threadIdx.x;
  const int nn = ne * P3;
  for (int q = t; q < P * P; q += kBatchThreads) sd[q] = dmat[q];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const T* src = fp[f] + e0 * P3;
    for (int q = t; q < nn; q += kBatchThreads) tiles[f * nn + q] = src[q];
  }
  __syncthreads();
  int bad = 0;
  T qkeep[MAXQ];
#pragma unroll
  for (int r = 0; r < MAXQ; ++r) {
    const int q = t + r * kBatchThreads;
    qkeep[r] = neg_inf<T>();
    if (q >= nn) continue;
    const int c = q / P3, node = q - c * P3;
    const int i = node % P, j = (node / P) % P, k = node / (P * P);
    const T* tl[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) tl[f] = tiles + f * nn + c * P3;
    T xr, xs, xt, yr, ys, yt, zr, zs, zt;
    ref_derivs<N>(tl[0], sd, i, j, k, xr, xs, xt);
    ref_derivs<N>(tl[1], sd, i, j, k, yr, ys, yt);
    ref_derivs<N>(tl[2], sd, i, j, k, zr, zs, zt);
    InvJac<T> kk;
    bad |= !invert_jacobian(xr, xs, xt, yr, ys, yt, zr, zs, zt, kk);
    T a[3][3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      T fr, fs, ft;
      ref_derivs<N>(tl[3 + cc], sd, i, j, k, fr, fs, ft);
      a[cc][0] = fr * kk.rx + fs * kk.sx + ft * kk.tx;
      a[cc][1] = fr * kk.ry + fs * kk.sy + ft * kk.ty;
      a[cc][2] = fr * kk.rz + fs * kk.sz + ft * kk.tz;
    }
    const T tr2 = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2] +
                  T(2) * (a[0][1] * a[1][0] + a[0][2] * a[2][0] + a[1][2] * a[2][1]);
    const T w1 = a[2][1] - a[1][2], w2 = a[0][2] - a[2][0], w3 = a[1][0] - a[0][1];
    const T qv = T(-0.5) * tr2;
    const int64_t o = e0 * P3 + q;
    if (oq) oq[o] = qv;
    if (oom) oom[o] = vort_root(w1 * w1 + w2 * w2 + w3 * w3);
    qkeep[r] = qv != qv ? neg_inf<T>() : qv;
    // one node at a time: no overlap of the unrolled iterations (which
    // would multiply the live registers)
    asm volatile("" ::: "memory");
  }
  if (oqmm) {
    __syncthreads();                     // every tile read is done
#pragma unroll
    for (int r = 0; r < MAXQ; ++r) {
      const int q = t + r * kBatchThreads;
      if (q < nn) tiles[q] = qkeep[r];
    }
    __syncthreads();
    const int wv = t >> 6, lane = t & 63;
    if (wv < ne) {                       // wave c reduces element c
      T mn = pos_inf<T>(), mx = neg_inf<T>();
      for (int q = lane; q < P3; q += 64) {
        const T v = tiles[wv * P3 + q];
        mn = v < mn ? v : mn;
        mx = v > mx ? v : mx;
      }
      wave_minmax(mn, mx);
      if (lane == 63) {
        oqmm[2 * (e0 + wv)] = mn;
        oqmm[2 * (e0 + wv) + 1] = mx;
      }
    }
  }
  return bad;
}

// A descriptor field read inside the persistent loop comes through vector
// loads (the loop's stores precede it); moving it to a scalar register keeps
// every pointer and address computation off the VGPRs.
template <typename P>
__device__ __forceinline__ P* uniform_ptr(P* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<P*>(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int64_t uniform_i64(int64_t x) {
  const uint64_t v = (uint64_t)x;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// One instantiation per (order, precision, form), so that no form's register
// demand limits another's occupancy.  kBatchNodeTile and kBatchDma7 run the
// per-element bodies of qcrit_tile and qcount_dma7 on one element per work
// item, kBatchPencil the body of qcrit_pencil on its workgroup's elements.
template <int N, typename T, int FORM>
constexpr int batch_threads() {
  return FORM == kBatchPencil     ? pencil_threads<N, T>()
         : FORM == kBatchNodeTile ? Shape<N>::kNodeThreads
                                  : kBatchThreads;
}

template <int N, typename T, int FORM>
__global__ void __launch_bounds__((batch_threads<N, T, FORM>()))
qcrit_batch(const BatchHeader* __restrict__ hdr, const BatchSnap* __restrict__ snaps,
            int32_t* __restrict__ status) {
  const int s0 = hdr->snap_begin[N], s1 = hdr->snap_begin[N + 1];
  const int64_t total = hdr->items[N];
  int bad = 0;
  // The descriptor of the current snapshot stays in scalar registers; a
  // workgroup's items increase, so it is looked up again only when an item
  // passes the next snapshot's first item.
  int cur = s0 - 1;
  int64_t begin = 0, next_begin = 0, n_elem = 0;
  int chunk = 1;
  const coef_t<N, T>* dmat = nullptr;
  const double* eo = nullptr;
  const T *f0 = nullptr, *f1 = nullptr, *f2 = nullptr, *f3 = nullptr, *f4 = nullptr,
          *f5 = nullptr;
  T *oq = nullptr, *oom = nullptr, *oqmm = nullptr;
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    if (cur < s0 || item >= next_begin) {
      int lo = cur < s0 ? s0 : cur, hi = s1 - 1;   // last snapshot with item_begin <= item
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (snaps[mid].item_begin <= item) lo = mid;
        else hi = mid - 1;
      }
      cur = __builtin_amdgcn_readfirstlane(lo);
      const BatchSnap& sn = snaps[cur];
      begin = uniform_i64(sn.item_begin);
      next_begin = uniform_i64(cur + 1 < s1 ? snaps[cur + 1].item_begin : total);
      n_elem = uniform_i64(sn.n_elem);
      chunk = __builtin_amdgcn_readfirstlane(sn.chunk);
      dmat = uniform_ptr(static_cast<const coef_t<N, T>*>(sn.dmat));
      eo = uniform_ptr(static_cast<const double*>(sn.eo));
      f0 = uniform_ptr(static_cast<const T*>(sn.f[0]));
      f1 = uniform_ptr(static_cast<const T*>(sn.f[1]));
      f2 = uniform_ptr(static_cast<const T*>(sn.f[2]));
      f3 = uniform_ptr(static_cast<const T*>(sn.f[3]));
      f4 = uniform_ptr(static_cast<const T*>(sn.f[4]));
      f5 = uniform_ptr(static_cast<const T*>(sn.f[5]));
      oq = uniform_ptr(static_cast<T*>(sn.q));
      oom = uniform_ptr(static_cast<T*>(sn.om));
      oqmm = uniform_ptr(static_cast<T*>(sn.qmm));
    }
    const int64_t e0 = (item - begin) * chunk;
    // the thread index is made opaque per item, so that no index arithmetic
    // of the body is hoisted out of the loop and held in registers across it
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    if constexpr (FORM == kBatchChunk) {
      __shared__ T tiles[kBatchTile];
      __shared__ coef_t<N, T> sd[(N + 1) * (N + 1)];
      const int64_t left = n_elem - e0;
      const int ne = (int)(left < chunk ? left : chunk);
      const T* fp[6] = {f0, f1, f2, f3, f4, f5};
      bad |= batch_chunk<N, T>(dmat, fp, oq, oom, oqmm, e0, ne, tiles, sd);
    } else if constexpr (FORM == kBatchNodeTile) {
      qcrit_tile_elem<N, T>(e0, t, dmat, f0, f1, f2, f3, f4, f5, oq, oom, oqmm, status);
    } else if constexpr (FORM == kBatchPencil) {
      constexpr int E = pencil_elems<N, T>();   // the item's chunk
      const int64_t left = n_elem - e0;
      const int ne = (int)(left < E ? left : E);
      qcrit_pencil_elem<N, T, false, E>(e0, t, dmat, f0, f1, f2, f3, f4, f5, oq, oom, oqmm,
                                        status, nullptr, ne);
    } else {
      static_assert(N == 7 && std::is_same<T, double>::value, "direct-to-LDS form: N = 7, FP64");
      qcount_dma7_elem<false>(e0, t, 0, eo, f0, f1, f2, f3, f4, f5, oq, oom, oqmm, 0,
                              IsoList<double>{}, nullptr, nullptr, nullptr, status);
    }
    __syncthreads();                   // the next item reuses the LDS
  }
  if constexpr (FORM == kBatchChunk) {
    bad = __syncthreads_or(bad);
    if (bad && threadIdx.x == 0 && status) atomicOr(status, SEM_FLAG_BAD_JACOBIAN);
  }
}

// ---------------------------------------------------------------------------
// batched isosurfaces: persistent count and emission over (job, element)
// ---------------------------------------------------------------------------
//
// A job is one field of one snapshot at up to four isovalues.  The plan
// lists the jobs grouped by order; within an order, work item k is element
// k - item_begin of the job whose item range holds k.  Count slots of a job
// are [slot_begin, slot_begin + n_iso * n_elem), isovalue-major, so one
// exclusive scan over every slot of every job gives each (job, isovalue,
// element) its first triangle in one soup ordered by job, isovalue,
// element, cell and slot.

// Isovalues read through a pointer (the job descriptor's copy).
template <typename T>
struct IsoPtr {
  const T* v;
};

// One soup with global offsets (the per-isovalue form of IsoOut is never
// taken, so nothing is indexed by isovalue).
template <typename T>
struct SoupOut {
  T* ptr[1];
  int64_t cap[1];
  static constexpr int per_iso = 0;
};

template <typename T>
__device__ __forceinline__ const T* job_iso(const IsoBatchJob& jb);
template <>
__device__ __forceinline__ const double* job_iso<double>(const IsoBatchJob& jb) {
  return jb.isod;
}
template <>
__device__ __forceinline__ const float* job_iso<float>(const IsoBatchJob& jb) {
  return jb.isof;
}

// The job descriptor a workgroup is in, kept in scalar registers and looked
// up again (binary search over the jobs' first items) only when the work
// item passes the next job's first item.
template <typename T>
struct JobCursor {
  int cur = -1;
  int64_t begin = 0, next_begin = 0, n_elem = 0, slot = 0;
  int n_iso = 0, job = 0;
  const T *x = nullptr, *y = nullptr, *z = nullptr, *field = nullptr, *mm = nullptr;
  const T* iso = nullptr;

  __device__ __forceinline__ void seek(const IsoBatchJob* __restrict__ jobs, int j0, int j1,
                                       int64_t total, int64_t item) {
    if (cur >= j0 && item < next_begin) return;
    int lo = cur < j0 ? j0 : cur, hi = j1 - 1;   // last job with item_begin <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (jobs[mid].item_begin <= item) lo = mid;
      else hi = mid - 1;
    }
    cur = __builtin_amdgcn_readfirstlane(lo);
    const IsoBatchJob& jb = jobs[cur];
    begin = uniform_i64(jb.item_begin);
    next_begin = uniform_i64(cur + 1 < j1 ? jobs[cur + 1].item_begin : total);
    n_elem = uniform_i64(jb.n_elem);
    slot = uniform_i64(jb.slot_begin);
    n_iso = __builtin_amdgcn_readfirstlane(jb.n_iso);
    job = __builtin_amdgcn_readfirstlane(jb.job);
    x = uniform_ptr(static_cast<const T*>(jb.x));
    y = uniform_ptr(static_cast<const T*>(jb.y));
    z = uniform_ptr(static_cast<const T*>(jb.z));
    field = uniform_ptr(static_cast<const T*>(jb.field));
    mm = uniform_ptr(static_cast<const T*>(jb.mm));
    iso = uniform_ptr(job_iso<T>(jb));
  }
};

template <int N, typename T>
__global__ void __launch_bounds__(128)
iso_batch_count(const IsoBatchHeader* __restrict__ hdr, const IsoBatchJob* __restrict__ jobs,
                const uint8_t* __restrict__ ntri_tab, int32_t* __restrict__ cnt,
                int64_t* __restrict__ active) {
  const int j0 = hdr->job_begin[N], j1 = hdr->job_begin[N + 1];
  const int64_t total = hdr->items[N];
  JobCursor<T> c;
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    c.seek(jobs, j0, j1, total, item);
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    count_elem<N, T>(item - c.begin, t, c.n_elem, c.field, c.mm, c.n_iso, IsoPtr<T>{c.iso},
                     ntri_tab, cnt + c.slot, active ? active + 4 * c.job : nullptr, nullptr);
    __syncthreads();                   // the next item reuses the LDS
  }
}

template <int N, typename T>
__global__ void __launch_bounds__(128)
iso_batch_emit(const IsoBatchHeader* __restrict__ hdr, const IsoBatchJob* __restrict__ jobs,
               const uint8_t* __restrict__ ntri_tab, const int32_t* __restrict__ cnt,
               const int64_t* __restrict__ offs, T* __restrict__ tri, int64_t cap) {
  const int j0 = hdr->job_begin[N], j1 = hdr->job_begin[N + 1];
  const int64_t total = hdr->items[N];
  SoupOut<T> out;
  out.ptr[0] = tri;
  out.cap[0] = cap;
  JobCursor<T> c;
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    c.seek(jobs, j0, j1, total, item);
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    emit_elem<N, T>(item - c.begin, t, c.n_elem, c.x, c.y, c.z, c.field, c.n_iso,
                    IsoPtr<T>{c.iso}, out, ntri_tab, cnt + c.slot, offs + c.slot, nullptr);
    __syncthreads();
  }
}

// Per (job, isovalue): first triangle and count (isovalues past a job's
// n_iso get count 0 at the job's end); the overflow flag if the soup does
// not fit.
__global__ void __launch_bounds__(256)
iso_batch_totals(const IsoBatchHeader* __restrict__ hdr, const IsoBatchJob* __restrict__ jobs,
                 const int64_t* __restrict__ offs, int64_t* __restrict__ tri_offset,
                 int64_t* __restrict__ tri_count, int64_t cap, int32_t* __restrict__ status) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx < 4 * hdr->n_job) {
    const IsoBatchJob& jb = jobs[idx >> 2];
    const int s = idx & 3;
    const int64_t lo = jb.slot_begin + (int64_t)(s < jb.n_iso ? s : jb.n_iso) * jb.n_elem;
    const int64_t hi = s < jb.n_iso ? lo + jb.n_elem : lo;
    if (tri_offset) tri_offset[4 * jb.job + s] = offs[lo];
    tri_count[4 * jb.job + s] = offs[hi] - offs[lo];
  }
  if (idx == 0 && status && offs[hdr->n_slots] > cap) atomicOr(status, SEM_FLAG_TRI_OVERFLOW);
}

__global__ void __launch_bounds__(256) fill_i64_n(int64_t* __restrict__ p, int64_t n,
                                                  int64_t value) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = value;
}

// Synthetic unit-cube elements on a 16 x 16 x ... lattice with node
// spacing 1/N and a smooth velocity: timing input for the autotuner.
template <typename T>
__global__ void tune_fill(int order, int64_t n_elem, T* x, T* y, T* z, T* u, T* v, T* w) {
  const int p = order + 1;
  const int64_t p3 = (int64_t)p * p * p;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n_elem * p3) return;
  const int64_t e = idx / p3;
  const int node = (int)(idx - e * p3);
  const int i = node % p, j = (node / p) % p, k = node / (p * p);
  const T xv = T(e % 16) + T(i) / T(order), yv = T((e / 16) % 16) + T(j) / T(order);
  const T zv = T(e / 256) + T(k) / T(order);
  x[idx] = xv;
  y[idx] = yv;
  z[idx] = zv;
  u[idx] = sin(xv + T(2) * yv);
  v[idx] = cos(yv - zv);
  w[idx] = sin(zv + T(0.5) * xv);
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

// D and its even-odd halves in the line sums' type of (order, T).
template <int N, typename T>
const coef_t<N, T>* dmat_of(const DeviceTables& tab) {
  if constexpr (std::is_same<coef_t<N, T>, float>::value) return tab.d32[N];
  else return tab.d64[N];
}

template <typename T>
hipError_t derivs_t(int order, const DeviceTables& tab, int64_t n_elem, const void* x,
                    const void* y, const void* z, const void* f, void* gx, void* gy, void* gz,
                    int32_t* status, hipStream_t s) {
  SEM_ORDER_SWITCH(order, {
    if constexpr (N <= 7) {
      hipLaunchKernelGGL((derivs_pencil<N, T>), dim3((unsigned)n_elem), dim3(Pen<N>::TH), 0, s, dmat_of<N, T>(tab),
                         (const T*)x, (const T*)y, (const T*)z, (const T*)f, (T*)gx, (T*)gy,
                         (T*)gz, status);
    } else {
      hipLaunchKernelGGL((derivs_tile<N, T>), dim3((unsigned)n_elem),
                         dim3(Shape<N>::kNodeThreads), 0, s, dmat_of<N, T>(tab), (const T*)x, (const T*)y,
                         (const T*)z, (const T*)f, (T*)gx, (T*)gy, (T*)gz, status);
    }
  });
  return hipGetLastError();
}

template <typename T>
hipError_t qcrit_t(int order, const DeviceTables& tab, int64_t n_elem, const void* x,
                   const void* y, const void* z, const void* u, const void* v, const void* w,
                   void* q, void* om, void* qmm, int32_t* status, hipStream_t s) {
  const PhaseTimer pt = phase_timer(SEM_PHASE_QCRIT);
  bool done = false;
  if constexpr (std::is_same<T, double>::value) {
    if (order == 7) {
      hipExtLaunchKernelGGL(qcount_dma7<false>, dim3((unsigned)n_elem), dim3(256), 0, s,
                            pt.start, pt.stop, 0, n_elem, tab.eo7, (const T*)x, (const T*)y,
                            (const T*)z, (const T*)u, (const T*)v, (const T*)w, (T*)q, (T*)om,
                            (T*)qmm, 0, IsoList<double>{}, (const uint8_t*)nullptr,
                            (int32_t*)nullptr, (int64_t*)nullptr, status);
      done = true;
    }
  }
  if (!done) {
    SEM_ORDER_SWITCH(order, {
      // pencil form wherever it is the faster one: every order in FP32,
      // N <= 7 in FP64 (at N = 8, 9 its FP64 registers spill)
      if constexpr (N <= 7 || !std::is_same<T, double>::value) {
        constexpr int E = (pencil_elems<N, T>());
        hipExtLaunchKernelGGL((qcrit_pencil<N, T>), dim3((unsigned)((n_elem + E - 1) / E)),
                              dim3(pencil_threads<N, T>()), 0, s, pt.start, pt.stop, 0, dmat_of<N, T>(tab),
                              (const T*)x, (const T*)y, (const T*)z, (const T*)u, (const T*)v,
                              (const T*)w, (T*)q, (T*)om, (T*)qmm, status, n_elem);
      } else {
        hipExtLaunchKernelGGL((qcrit_tile<N, T>), dim3((unsigned)n_elem),
                              dim3(Shape<N>::kNodeThreads), 0, s, pt.start, pt.stop, 0, dmat_of<N, T>(tab),
                              (const T*)x, (const T*)y, (const T*)z, (const T*)u, (const T*)v,
                              (const T*)w, (T*)q, (T*)om, (T*)qmm, status);
      }
    });
  }
  phase_done(pt);
  return hipGetLastError();
}

bool is_mixed(sem_dtype dt) {
  return dt == SEM_MIXED_BF16 || dt == SEM_MIXED_FP16 || dt == SEM_MIXED_BF16X3 ||
         dt == SEM_MIXED_FP16X3;
}

// Mixed-precision kernels (N = 7, FP32 storage).  QC: Q / |omega| / range
// into (o0, o1, qmm); otherwise the gradient of u into (o0, o1, o2).
template <bool QC>
hipError_t mixed_t(sem_dtype dt, const DeviceTables& tab, int64_t n_elem, const void* x,
                   const void* y, const void* z, const void* u, const void* v, const void* w,
                   void* o0, void* o1, void* o2, void* qmm, int32_t* status, hipStream_t s,
                   const PhaseTimer& pt, const CountSink<float>* sink = nullptr) {
  const CountSink<float> none{};
  const CountSink<float>& sk = sink ? *sink : none;
  auto go = [&](auto kern) {
    hipExtLaunchKernelGGL(kern, dim3((unsigned)n_elem), dim3(256), 0, s, pt.start, pt.stop, 0,
                          tab.d64[7], (const float*)x, (const float*)y, (const float*)z,
                          (const float*)u, (const float*)v, (const float*)w, (float*)o0,
                          (float*)o1, (float*)o2, (float*)qmm, status, sk);
  };
  constexpr bool kC = QC;   // counting variants exist with Q only
  switch (dt) {
    case SEM_MIXED_BF16:
      sink ? go(mixed7<kMixBF16, QC, kC>) : go(mixed7<kMixBF16, QC>);
      break;
    case SEM_MIXED_FP16:
      sink ? go(mixed7<kMixFP16, QC, kC>) : go(mixed7<kMixFP16, QC>);
      break;
    case SEM_MIXED_BF16X3:
      sink ? go(mixed7<kMixBF16x3, QC, kC>) : go(mixed7<kMixBF16x3, QC>);
      break;
    case SEM_MIXED_FP16X3:
      sink ? go(mixed7<kMixFP16x3, QC, kC>) : go(mixed7<kMixFP16x3, QC>);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
IsoList<T> make_isolist(int n_iso, const double* iso_host) {
  IsoList<T> iso;
  for (int q = 0; q < SEM_MAX_ISO; ++q) iso.v[q] = q < n_iso ? (T)iso_host[q] : T(0);
  return iso;
}

// Scan of the per-(isovalue, element) counts, totals, then emission.
// Exclusive scan of count int32 values into offs[0..count]: tile sums,
// then the tiles' offsets (folded into the apply kernel when there are at
// most kScanFold tiles, else through a one-workgroup scan of the sums).
// Tiles of 1,024 counts up to kScanSmall counts (always folded), else of
// 4,096 (scan_tile).  `start` and `stop` (may be null) stamp the first and
// the last kernel.
template <int ITEMS>
void scan_kernels_t(const int32_t* cnt, int64_t count, int64_t* partial, int64_t* offs,
                    hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  static_assert(kScanThreads * ITEMS == 1024 || kScanThreads * ITEMS == 4096, "scan_tile");
  const int64_t nb = scan_blocks(count);
  hipExtLaunchKernelGGL(scan_reduce<ITEMS>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, start,
                        nullptr, 0, cnt, count, partial);
  if (nb <= kScanFold) {
    hipExtLaunchKernelGGL((scan_apply<true, ITEMS>), dim3((unsigned)nb), dim3(kScanThreads), 0,
                          s, nullptr, stop, 0, cnt, count, (const int64_t*)partial, nb, offs);
  } else {
    hipLaunchKernelGGL(scan_partials, dim3(1), dim3(1024), 0, s, partial, nb);
    hipExtLaunchKernelGGL((scan_apply<false, ITEMS>), dim3((unsigned)nb), dim3(kScanThreads), 0,
                          s, nullptr, stop, 0, cnt, count, (const int64_t*)partial, nb, offs);
  }
}
void scan_kernels(const int32_t* cnt, int64_t count, int64_t* partial, int64_t* offs,
                  hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  if (scan_tile(count) == 1024)
    scan_kernels_t<1024 / kScanThreads>(cnt, count, partial, offs, s, start, stop);
  else
    scan_kernels_t<4096 / kScanThreads>(cnt, count, partial, offs, s, start, stop);
}

template <typename T>
hipError_t iso_scan_emit(int order, const DeviceTables& tab, int64_t n_elem, const void* x,
                         const void* y, const void* z, const void* field, int n_iso,
                         const IsoList<T>& iso, const IsoOut<T>& out, uint64_t* keys,
                         int64_t* tri_count, const IsoWorkspace& ws, int32_t* status,
                         hipStream_t s) {
  const int64_t count = (int64_t)n_iso * n_elem;
  const PhaseTimer ps = phase_timer(SEM_PHASE_SCAN);
  scan_kernels(ws.cnt, count, ws.partial, ws.offs, s, ps.start, ps.stop);
  phase_done(ps);
  bool any_cap = false;
  for (int q = 0; q < (out.per_iso ? n_iso : 1); ++q) any_cap = any_cap || out.cap[q] > 0;
  // the totals: a kernel of their own, unless the emission kernel for odd
  // orders writes them
  if (!any_cap || order % 2 == 0)
    hipLaunchKernelGGL((iso_totals<T>), dim3(1), dim3(SEM_MAX_ISO), 0, s, (const int64_t*)ws.offs,
                       n_elem, n_iso, tri_count, out, status);
  if (!any_cap) return hipGetLastError();
  const PhaseTimer pe = phase_timer(SEM_PHASE_EMIT);
  SEM_ORDER_SWITCH(order, {
    if constexpr (N % 2 == 1) {
      hipExtLaunchKernelGGL((emit_direct<N, T>), dim3((unsigned)n_elem), dim3(128), 0, s,
                            pe.start, pe.stop, 0, n_elem, (const T*)x, (const T*)y,
                            (const T*)z, (const T*)field, n_iso, iso, out, tab.ntri,
                            (const int32_t*)ws.cnt, (const int64_t*)ws.offs, keys, tri_count,
                            status);
    } else {
      hipExtLaunchKernelGGL((iso_emit<N, T>), dim3((unsigned)n_elem),
                            dim3(Shape<N>::kCellThreads), 0, s, pe.start, pe.stop, 0, n_elem,
                            (const T*)x, (const T*)y, (const T*)z, (const T*)field, n_iso, iso,
                            tab.ntri, tab.tri, (const int32_t*)ws.cnt, (const int64_t*)ws.offs,
                            out, keys);
    }
  });
  phase_done(pe);
  return hipGetLastError();
}

// Two-pass isosurface of a given field: count, exclusive scan, emit.
template <typename T>
hipError_t iso_pipeline(int order, const DeviceTables& tab, int64_t n_elem, const void* x,
                        const void* y, const void* z, const void* field, const void* mm,
                        int n_iso, const double* iso_host, const IsoOut<T>& out,
                        uint64_t* keys, int64_t* tri_count, int64_t* active,
                        uint8_t* case_idx, const IsoWorkspace& ws, int32_t* status,
                        hipStream_t s) {
  const IsoList<T> iso = make_isolist<T>(n_iso, iso_host);
  if (active) hipLaunchKernelGGL(fill_i64, dim3(1), dim3(64), 0, s, active, n_iso, (int64_t)0);
  const PhaseTimer pt = phase_timer(SEM_PHASE_COUNT);
  SEM_ORDER_SWITCH(order, {
    if constexpr (N % 2 == 1) {
      hipExtLaunchKernelGGL((count_direct<N, T>), dim3((unsigned)n_elem), dim3(128), 0, s,
                            pt.start, pt.stop, 0, n_elem, (const T*)field, (const T*)mm, n_iso,
                            iso, tab.ntri, ws.cnt, active, case_idx);
    } else {
      hipExtLaunchKernelGGL((iso_count<N, T>), dim3((unsigned)n_elem),
                            dim3(Shape<N>::kCellThreads), 0, s, pt.start, pt.stop, 0, n_elem,
                            (const T*)field, (const T*)mm, n_iso, iso, tab.ntri, ws.cnt, active,
                            case_idx);
    }
  });
  phase_done(pt);
  return iso_scan_emit<T>(order, tab, n_elem, x, y, z, field, n_iso, iso, out, keys, tri_count,
                          ws, status, s);
}

template <typename T>
hipError_t iso_t(int order, const DeviceTables& tab, int64_t n_elem, const void* x,
                 const void* y, const void* z, const void* field, const void* mm, int n_iso,
                 const double* iso_host, void* tri_xyz, int64_t cap, uint64_t* keys,
                 int64_t* tri_count, int64_t* active, uint8_t* case_idx,
                 const IsoWorkspace& ws, int32_t* status, hipStream_t s) {
  IsoOut<T> out{};
  out.ptr[0] = static_cast<T*>(tri_xyz);
  out.cap[0] = cap;
  out.per_iso = 0;
  return iso_pipeline<T>(order, tab, n_elem, x, y, z, field, mm, n_iso, iso_host, out, keys,
                         tri_count, active, case_idx, ws, status, s);
}

// sem_extract: q and qmm always point at storage (the caller's or the
// workspace's); `ws` is the isosurface part of the workspace.
template <typename T>
hipError_t extract_t(int order, sem_dtype dt, const DeviceTables& tab, int64_t n_elem,
                     const void* x,
                     const void* y, const void* z, const void* u, const void* v,
                     const void* w, void* q, void* om, void* qmm, int n_iso,
                     const double* iso_host, void* const* tri_xyz, const int64_t* cap,
                     int64_t* tri_count, int64_t* active, const IsoWorkspace& ws,
                     int32_t* status, hipStream_t s) {
  IsoOut<T> out{};
  for (int k = 0; k < n_iso; ++k) {
    out.ptr[k] = static_cast<T*>(tri_xyz[k]);
    out.cap[k] = cap[k];
  }
  out.per_iso = 1;
  const IsoList<T> iso = make_isolist<T>(n_iso, iso_host);
  if constexpr (std::is_same<T, double>::value) {
    if (order == 7) {
      if (active)
        hipLaunchKernelGGL(fill_i64, dim3(1), dim3(64), 0, s, active, n_iso, (int64_t)0);
      const PhaseTimer pt = phase_timer(SEM_PHASE_QCRIT);
      hipExtLaunchKernelGGL(qcount_dma7<true>, dim3((unsigned)n_elem), dim3(256), 0, s,
                            pt.start, pt.stop, 0, n_elem, tab.eo7, (const T*)x, (const T*)y,
                            (const T*)z, (const T*)u, (const T*)v, (const T*)w, (T*)q, (T*)om,
                            (T*)qmm, n_iso, iso, tab.ntri, ws.cnt, active, status);
      phase_done(pt);
      return iso_scan_emit<T>(order, tab, n_elem, x, y, z, q, n_iso, iso, out, nullptr,
                              tri_count, ws, status, s);
    }
  }
  hipError_t err;
  bool fused = false;
  if (!is_mixed(dt)) {
    // pencil forms (sem_qcrit's choice: every order in FP32, N <= 6 in FP64
    // here) count in the Q kernel
    CountSink<T> sink;
    sink.n_iso = n_iso;
    sink.iso = iso;
    sink.ntri = tab.ntri;
    sink.cnt = ws.cnt;
    sink.active = active;
    sink.n_elem = n_elem;
    SEM_ORDER_SWITCH(order, {
      if constexpr (N <= 7 || !std::is_same<T, double>::value) {
        if (active)
          hipLaunchKernelGGL(fill_i64, dim3(1), dim3(64), 0, s, active, n_iso, (int64_t)0);
        const PhaseTimer pt = phase_timer(SEM_PHASE_QCRIT);
        constexpr int E = (pencil_elems<N, T>());
        hipExtLaunchKernelGGL((qcount_pencil<N, T>), dim3((unsigned)((n_elem + E - 1) / E)),
                              dim3(pencil_threads<N, T>()), 0, s, pt.start, pt.stop, 0, dmat_of<N, T>(tab),
                              (const T*)x, (const T*)y,
                              (const T*)z, (const T*)u, (const T*)v, (const T*)w, (T*)q,
                              (T*)om, (T*)qmm, status, sink);
        phase_done(pt);
        fused = true;
      }
    });
  }
  if (fused) {
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    return iso_scan_emit<T>(order, tab, n_elem, x, y, z, q, n_iso, iso, out, nullptr,
                            tri_count, ws, status, s);
  }
  if (is_mixed(dt)) {
    if constexpr (std::is_same<T, float>::value) {
      if (active)
        hipLaunchKernelGGL(fill_i64, dim3(1), dim3(64), 0, s, active, n_iso, (int64_t)0);
      CountSink<float> sink;
      sink.n_iso = n_iso;
      sink.iso = iso;
      sink.ntri = tab.ntri;
      sink.cnt = ws.cnt;
      sink.active = active;
      sink.n_elem = n_elem;
      const PhaseTimer pt = phase_timer(SEM_PHASE_QCRIT);
      err = mixed_t<true>(dt, tab, n_elem, x, y, z, u, v, w, q, om, nullptr, qmm, status, s, pt,
                          &sink);
      phase_done(pt);
      if (err != hipSuccess) return err;
      return iso_scan_emit<T>(order, tab, n_elem, x, y, z, q, n_iso, iso, out, nullptr,
                              tri_count, ws, status, s);
    }
    const PhaseTimer pt = phase_timer(SEM_PHASE_QCRIT);
    err = mixed_t<true>(dt, tab, n_elem, x, y, z, u, v, w, q, om, nullptr, qmm, status, s, pt);
    phase_done(pt);
  } else {
    err = qcrit_t<T>(order, tab, n_elem, x, y, z, u, v, w, q, om, qmm, status, s);
  }
  if (err != hipSuccess) return err;
  return iso_pipeline<T>(order, tab, n_elem, x, y, z, q, qmm, n_iso, iso_host, out, nullptr,
                         tri_count, active, nullptr, ws, status, s);
}

}  // namespace

int64_t scan_blocks(int64_t count) { return scan_tiles(count); }

size_t batch_plan_bytes(int n_snap) {
  return 256 + (((size_t)n_snap * sizeof(BatchSnap) + 255) & ~size_t(255));
}

int batch_variant_chunk(int order, sem_dtype dt, int variant) {
  if (variant < 3) return 1 << variant;
  return batch_variant_form(variant) == kBatchPencil ? pencil_elems_of(order, dt == SEM_F64) : 1;
}

int batch_variant_form(int variant) {
  static const int form[kBatchVariants] = {kBatchChunk, kBatchChunk, kBatchChunk, kBatchPencil,
                                           kBatchDma7, kBatchNodeTile};
  return form[variant];
}

bool batch_variant_ok(int order, sem_dtype dt, int variant) {
  if (variant < 0 || variant >= kBatchVariants) return false;
  if (order < 1 || order > kMaxOrder) return false;
  const int p3 = (order + 1) * (order + 1) * (order + 1);
  switch (batch_variant_form(variant)) {
    case kBatchChunk: return batch_variant_chunk(order, dt, variant) * p3 <= kBatchTile / 6;
    case kBatchPencil: return true;
    case kBatchNodeTile: return true;
    default: return order == 7 && dt == SEM_F64;
  }
}

// untuned: the form sem_qcrit itself uses for this order and precision
int batch_default_variant(int order, sem_dtype dt) {
  if (order == 7 && dt == SEM_F64) return 4;
  return (order <= 7 || dt == SEM_F32) ? 3 : 5;
}

template <int N, typename T>
const void* batch_kernel_nt(int form) {
  if (form == kBatchPencil)
    return reinterpret_cast<const void*>(&qcrit_batch<N, T, kBatchPencil>);
  if constexpr (N == 7 && std::is_same<T, double>::value) {
    if (form == kBatchDma7)
      return reinterpret_cast<const void*>(&qcrit_batch<7, double, kBatchDma7>);
  }
  if (form == kBatchNodeTile)
    return reinterpret_cast<const void*>(&qcrit_batch<N, T, kBatchNodeTile>);
  return form == kBatchChunk ? reinterpret_cast<const void*>(&qcrit_batch<N, T, kBatchChunk>)
                             : nullptr;
}

int batch_threads_of(int n, bool f64, int form) {
  if (form == kBatchPencil)
    return 128 * ((pencil_elems_of(n, f64) * (n + 1) * (n + 1) + 63) / 64);
  if (form == kBatchNodeTile) return (((n + 1) * (n + 1) * (n + 1) + 63) / 64) * 64;
  return kBatchThreads;
}

template <int N>
const void* batch_kernel_n(bool f64, int form) {
  return f64 ? batch_kernel_nt<N, double>(form) : batch_kernel_nt<N, float>(form);
}

const void* batch_kernel(int n, bool f64, int form) {
  switch (n) {
    case 1: return batch_kernel_n<1>(f64, form);
    case 2: return batch_kernel_n<2>(f64, form);
    case 3: return batch_kernel_n<3>(f64, form);
    case 4: return batch_kernel_n<4>(f64, form);
    case 5: return batch_kernel_n<5>(f64, form);
    case 6: return batch_kernel_n<6>(f64, form);
    case 7: return batch_kernel_n<7>(f64, form);
    case 8: return batch_kernel_n<8>(f64, form);
    case 9: return batch_kernel_n<9>(f64, form);
    default: return nullptr;
  }
}

// Workgroups of a persistent launch: every CU filled to the kernel's
// occupancy (queried once per kernel).
int batch_grid(const void* fn, int threads, int cu_count) {
  static std::mutex mu;
  static std::unordered_map<const void*, int> occ;
  std::lock_guard<std::mutex> lock(mu);
  auto it = occ.find(fn);
  if (it == occ.end()) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, threads, 0) != hipSuccess ||
        blocks < 1)
      blocks = 2;
    it = occ.emplace(fn, blocks).first;
  }
  return it->second * cu_count;
}

hipError_t launch_qcrit_batch(sem_dtype dt, const void* plan, unsigned launch_code, int cu_count,
                              int32_t* status, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const BatchHeader* hdr = static_cast<const BatchHeader*>(plan);
  const BatchSnap* snaps =
      reinterpret_cast<const BatchSnap*>(static_cast<const char*>(plan) + 256);
  int first = -1, last = -1;
  for (int n = 1; n <= kMaxOrder; ++n)
    if (launch_code_form(launch_code, n) >= 0) {
      if (first < 0) first = n;
      last = n;
    }
  if (first < 0) return hipSuccess;
  for (int n = first; n <= last; ++n) {
    const int form = launch_code_form(launch_code, n);
    if (form < 0) continue;
    const void* fn = batch_kernel(n, dt == SEM_F64, form);
    if (!fn) return hipErrorInvalidValue;
    hipEvent_t a = n == first ? e0 : nullptr, b = n == last ? e1 : nullptr;
    void* args[] = {const_cast<BatchHeader**>(&hdr), const_cast<BatchSnap**>(&snaps), &status};
    const int threads = batch_threads_of(n, dt == SEM_F64, form);
    const hipError_t err = hipExtLaunchKernel(fn, dim3(batch_grid(fn, threads, cu_count)),
                                              dim3(threads), args, 0, s, a, b, 0);
    if (err != hipSuccess) return err;
  }
  return hipGetLastError();
}

size_t iso_batch_plan_bytes(int n_job) {
  return 256 + (((size_t)n_job * sizeof(IsoBatchJob) + 255) & ~size_t(255));
}

namespace {
template <int N>
hipError_t iso_batch_phase(bool f64, bool emit, const IsoBatchHeader* hdr,
                           const IsoBatchJob* jobs, const DeviceTables& tab,
                           const IsoWorkspace& ws, int64_t* active, void* tri, int64_t cap,
                           hipStream_t s, hipEvent_t a, hipEvent_t b) {
  const void* fn;
  if (emit)
    fn = f64 ? reinterpret_cast<const void*>(&iso_batch_emit<N, double>)
             : reinterpret_cast<const void*>(&iso_batch_emit<N, float>);
  else
    fn = f64 ? reinterpret_cast<const void*>(&iso_batch_count<N, double>)
             : reinterpret_cast<const void*>(&iso_batch_count<N, float>);
  const uint8_t* ntri = tab.ntri;
  int32_t* cnt = ws.cnt;
  int64_t* offs = ws.offs;
  void* count_args[] = {&hdr, &jobs, &ntri, &cnt, &active};
  void* emit_args[] = {&hdr, &jobs, &ntri, &cnt, &offs, &tri, &cap};
  // Four times the workgroups the CUs hold at once: the cost of an element
  // varies with its triangles, and with a grid of exactly the resident
  // workgroups the unluckiest one sets the end (measured on the batched
  // benchmark snapshots: 4.54 ms at 1x, 3.58 at 4x, 3.60 at 16x, 3.84 at 64x;
  // 48 separate sem_isosurface calls: 4.4 ms).  Workgroups that start later
  // take the slots the early finishers free.
  return hipExtLaunchKernel(fn, dim3(4 * batch_grid(fn, 128, tab.cu_count)), dim3(128),
                            emit ? emit_args : count_args, 0, s, a, b, 0);
}
}  // namespace

hipError_t launch_iso_batch(sem_dtype dt, const DeviceTables& tab, const void* plan,
                            unsigned launch_code, int n_job, int64_t n_slots, void* tri,
                            int64_t cap, int64_t* tri_offset, int64_t* tri_count,
                            int64_t* active, const IsoWorkspace& ws, int32_t* status,
                            hipStream_t s) {
  const IsoBatchHeader* hdr = static_cast<const IsoBatchHeader*>(plan);
  const IsoBatchJob* jobs =
      reinterpret_cast<const IsoBatchJob*>(static_cast<const char*>(plan) + 256);
  const bool f64 = dt == SEM_F64;
  if (active && n_job > 0)
    hipLaunchKernelGGL(fill_i64_n, dim3((unsigned)((4 * (int64_t)n_job + 255) / 256)), dim3(256),
                       0, s, active, 4 * (int64_t)n_job, (int64_t)0);
  int first = -1, last = -1;
  for (int n = 1; n <= kMaxOrder; ++n)
    if (launch_code >> n & 1u) {
      if (first < 0) first = n;
      last = n;
    }
  for (int pass = 0; pass < 2; ++pass) {
    const PhaseTimer pt = phase_timer(pass == 0 ? SEM_PHASE_COUNT : SEM_PHASE_EMIT);
    for (int n = first; n >= 1 && n <= last; ++n) {
      if (!(launch_code >> n & 1u)) continue;
      hipEvent_t a = n == first ? pt.start : nullptr, b = n == last ? pt.stop : nullptr;
      hipError_t err = hipSuccess;
      switch (n) {
        case 1: err = iso_batch_phase<1>(f64, pass, hdr, jobs, tab, ws, active, tri, cap, s, a, b); break;
        case 2: err = iso_batch_phase<2>(f64, pass, hdr, jobs, tab, ws, active, tri, cap, s, a, b); break;
        case 3: err = iso_batch_phase<3>(f64, pass, hdr, jobs, tab, ws, active, tri, cap, s, a, b); break;
        case 4: err = iso_batch_phase<4>(f64, pass, hdr, jobs, tab, ws, active, tri, cap, s, a, b); break;
        case 5: err = iso_batch_phase<5>(f64, pass, hdr, jobs, tab, ws, active, tri, cap, s, a, b); break;
        case 6: err = iso_batch_phase<6>(f64, pass, hdr, jobs, tab, ws, active, tri, cap, s, a, b); break;
        case 7: err = iso_batch_phase<7>(f64, pass, hdr, jobs, tab, ws, active, tri, cap, s, a, b); break;
        case 8: err = iso_batch_phase<8>(f64, pass, hdr, jobs, tab, ws, active, tri, cap, s, a, b); break;
        case 9: err = iso_batch_phase<9>(f64, pass, hdr, jobs, tab, ws, active, tri, cap, s, a, b); break;
        default: err = hipErrorInvalidValue;
      }
      if (err != hipSuccess) return err;
    }
    phase_done(pt);
    if (pass == 0) {
      // one exclusive scan over every count slot, then the per-(job,
      // isovalue) totals
      const PhaseTimer ps = phase_timer(SEM_PHASE_SCAN);
      scan_kernels(ws.cnt, n_slots, ws.partial, ws.offs, s, ps.start, nullptr);
      const unsigned tb = (unsigned)((4 * (int64_t)n_job + 255) / 256);
      hipExtLaunchKernelGGL(iso_batch_totals, dim3(tb > 0 ? tb : 1), dim3(256), 0, s, nullptr,
                            ps.stop, 0, hdr, jobs, (const int64_t*)ws.offs, tri_offset,
                            tri_count, cap, status);
      phase_done(ps);
      if (cap <= 0) break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_tune_fill(sem_dtype dt, int order, int64_t n_elem, void* const* f,
                            hipStream_t s) {
  const int64_t p = order + 1, n = n_elem * p * p * p;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (dt == SEM_F64)
    hipLaunchKernelGGL(tune_fill<double>, dim3(blocks), dim3(256), 0, s, order, n_elem,
                       (double*)f[0], (double*)f[1], (double*)f[2], (double*)f[3],
                       (double*)f[4], (double*)f[5]);
  else
    hipLaunchKernelGGL(tune_fill<float>, dim3(blocks), dim3(256), 0, s, order, n_elem,
                       (float*)f[0], (float*)f[1], (float*)f[2], (float*)f[3], (float*)f[4],
                       (float*)f[5]);
  return hipGetLastError();
}

hipError_t launch_exclusive_scan(const int32_t* cnt, int64_t count, int64_t* partial,
                                 int64_t* offs, hipStream_t s) {
  scan_kernels(cnt, count, partial, offs, s, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_derivs(int order, sem_dtype dt, const DeviceTables& tab, int64_t n_elem,
                         const void* x, const void* y, const void* z, const void* f, void* gx,
                         void* gy, void* gz, int32_t* status, hipStream_t s) {
  if (is_mixed(dt))
    return mixed_t<false>(dt, tab, n_elem, x, y, z, f, nullptr, nullptr, gx, gy, gz, nullptr,
                          status, s, PhaseTimer{});
  return dt == SEM_F64 ? derivs_t<double>(order, tab, n_elem, x, y, z, f, gx, gy, gz, status, s)
                       : derivs_t<float>(order, tab, n_elem, x, y, z, f, gx, gy, gz, status, s);
}

hipError_t launch_qcrit(int order, sem_dtype dt, const DeviceTables& tab, int64_t n_elem,
                        const void* x, const void* y, const void* z, const void* u,
                        const void* v, const void* w, void* q, void* om, void* qmm,
                        int32_t* status, hipStream_t s) {
  if (is_mixed(dt)) {
    const PhaseTimer pt = phase_timer(SEM_PHASE_QCRIT);
    const hipError_t e =
        mixed_t<true>(dt, tab, n_elem, x, y, z, u, v, w, q, om, nullptr, qmm, status, s, pt);
    phase_done(pt);
    return e;
  }
  return dt == SEM_F64
             ? qcrit_t<double>(order, tab, n_elem, x, y, z, u, v, w, q, om, qmm, status, s)
             : qcrit_t<float>(order, tab, n_elem, x, y, z, u, v, w, q, om, qmm, status, s);
}

hipError_t launch_extract(int order, sem_dtype dt, const DeviceTables& tab, int64_t n_elem,
                          const void* x, const void* y, const void* z, const void* u,
                          const void* v, const void* w, void* q, void* om, void* qmm,
                          int n_iso, const double* iso_host, void* const* tri_xyz,
                          const int64_t* tri_capacity, int64_t* tri_count,
                          int64_t* active_cells, const IsoWorkspace& ws, int32_t* status,
                          hipStream_t s) {
  return dt == SEM_F64
             ? extract_t<double>(order, dt, tab, n_elem, x, y, z, u, v, w, q, om, qmm, n_iso,
                                 iso_host, tri_xyz, tri_capacity, tri_count, active_cells, ws,
                                 status, s)
             : extract_t<float>(order, dt, tab, n_elem, x, y, z, u, v, w, q, om, qmm, n_iso,
                                iso_host, tri_xyz, tri_capacity, tri_count, active_cells, ws,
                                status, s);
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
