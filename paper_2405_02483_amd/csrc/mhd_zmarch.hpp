// Building blocks of the z-marching kernels: each workgroup owns a TX x TY
// tile of (x, y) columns of one box and walks a range of z planes.  Stencils
// across x and y read LDS copies of the current plane (with halo); stencils
// along z read short per-thread register windows of past planes, or scatter
// a new plane's value into per-thread accumulators of the output planes it
// feeds.  A window slot m holds plane (base + m) in marching order
// (periodic planes are numbered without wrapping, so the slot of a plane is
// fixed at compile time); planes that do not exist on a wall-bounded axis
// hold 0 and get coefficient 0.
#pragma once

#include "mhd_kernels.hpp"

namespace smhd {

// One work item: a tile of columns and a range [z0, z1) of output planes.
struct ZItem {
  int box;
  int x0, y0;
  int z0, z1;
  int pad;
};

// Per-workgroup partial maxima for the Courant time step.
struct CPart {
  double cmax;     // max c_s + c_A + |u_perp|
  double numax;    // max speed-like viscosity
};

__device__ __forceinline__ int wrapm(int a, int n) {
  const int r = a % n;
  return r < 0 ? r + n : r;
}

// Coefficient of plane p in the output of plane k of a z operator on a
// wall-bounded axis of N planes (same order choice as opwall).
template <int FAM, int FORM, class T>
__device__ __forceinline__ T zcoef_wall(int k, int p, int N) {
  int c = k + FORM;
  int q = min(3, min(c, N - c));
  if (q == 0) {
    c = FORM ? N - 1 : 1;
    q = 1;
  }
  const int d = p - c;
  const int P = d >= 0 ? d + 1 : -d;
  if (P > q) return T(0);
  T w;
  if (q == 3) {
    w = FAM == 0 ? (P == 1 ? Cf<T>::IA : (P == 2 ? Cf<T>::IB : Cf<T>::IC))
                 : (P == 1 ? Cf<T>::DA : (P == 2 ? Cf<T>::DB : Cf<T>::DC));
  } else if (q == 2) {
    w = FAM == 0 ? (P == 1 ? Cf<T>::I4A : Cf<T>::I4B) : (P == 1 ? Cf<T>::D4A : Cf<T>::D4B);
  } else {
    w = FAM == 0 ? T(0.5) : T(1);
  }
  return (FAM == 1 && d < 0) ? -w : w;
}

// Sixth-order coefficient for offset d = p - k (periodic axis, or an output
// plane whose full stencil lies inside the array).
template <int FAM, int FORM, class T>
__device__ __forceinline__ constexpr T zcoef6(int d) {
  // pairs (c+P-1, c-P) with c = k + FORM
  const int dd = d - FORM;
  const int P = dd >= 0 ? dd + 1 : -dd;
  if (P > 3) return T(0);
  const T w = FAM == 0 ? (P == 1 ? Cf<T>::IA : (P == 2 ? Cf<T>::IB : Cf<T>::IC))
                       : (P == 1 ? Cf<T>::DA : (P == 2 ? Cf<T>::DB : Cf<T>::DC));
  return (FAM == 1 && dd < 0) ? -w : w;
}

// z operator at output plane q from a register window whose slot LAG holds
// plane q.  Periodic: the fixed sixth-order stencil; wall: coefficient per
// slot from the plane-dependent order.  FAM 0 interpolation, 1 derivative;
// FORM 0 dn, 1 up.
template <int FAM, int FORM, int W, int LAG, class T>
__device__ __forceinline__ T zwin(const T (&w)[W], int q, bool wall, int N, T hinv) {
  static_assert(LAG >= 3 - FORM && W - 1 - LAG >= 2 + FORM, "window too short");
  if (!wall) {
    return op6<FAM, FORM, T>([&](int m) { return w[LAG + m]; }, hinv);
  }
  T acc = T(0);
#pragma unroll
  for (int m = 0; m < W; ++m) acc += zcoef_wall<FAM, FORM, T>(q, q - LAG + m, N) * w[m];
  return FAM ? acc * hinv : acc;
}

template <int W, class T> __device__ __forceinline__ void push(T (&w)[W], T v) {
#pragma unroll
  for (int m = 0; m < W - 1; ++m) w[m] = w[m + 1];
  w[W - 1] = v;
}

// Scatter the value v of input plane p = kbase + PK into accumulators
// acc[s] of output planes k = kbase + s (s = 0..6) of a z operator (the 1/h
// of a derivative is folded into v by the caller).
template <int FAM, int FORM, int PK, class T>
__device__ __forceinline__ void zscatter(T (&acc)[7], int kbase, T v, bool wall, int N) {
  if (!wall) {
#pragma unroll
    for (int s = 0; s < 7; ++s) acc[s] += zcoef6<FAM, FORM, T>(PK - s) * v;
    return;
  }
#pragma unroll
  for (int s = 0; s < 7; ++s) {
    const int k = kbase + s;
    if (k >= 0 && k < N) acc[s] += zcoef_wall<FAM, FORM, T>(k, kbase + PK, N) * v;
  }
}

// Staggered derivative written on first differences d_m = f[m] - f[m-1]:
// with c = k + FORM and q pairs, f[c+P-1] - f[c-P] telescopes into the sum
// of d_m over |m - c| <= P - 1, so output k = sum_m W(k, m) d_m / h with
// W = sum of the pair coefficients d_P over P > |m - c|.  Scattering d_m
// (instead of f) keeps the rounding relative to the differences, as in the
// gather form, where a plain scatter of f would round relative to |f|.
template <int FORM, class T>
__device__ __forceinline__ T zdcoef_wall(int k, int m, int N) {
  int c = k + FORM;
  int q = min(3, min(c, N - c));
  if (q == 0) {
    c = FORM ? N - 1 : 1;
    q = 1;
  }
  const int j = m - c < 0 ? c - m : m - c;
  T w = T(0);
  if (q == 3) {
    if (j <= 0) w += Cf<T>::DA;
    if (j <= 1) w += Cf<T>::DB;
    if (j <= 2) w += Cf<T>::DC;
  } else if (q == 2) {
    if (j <= 0) w += Cf<T>::D4A;
    if (j <= 1) w += Cf<T>::D4B;
  } else {
    if (j == 0) w = T(1);
  }
  return w;
}

template <int FORM, class T>
__device__ __forceinline__ constexpr T zdcoef6(int d) {
  // d = m - k; j = |m - c| with c = k + FORM
  const int j = d - FORM < 0 ? FORM - d : d - FORM;
  return j == 0 ? Cf<T>::DA + Cf<T>::DB + Cf<T>::DC
                : (j == 1 ? Cf<T>::DB + Cf<T>::DC : (j == 2 ? Cf<T>::DC : T(0)));
}

// Scatter the first difference dv = f[p] - f[p-1] (times 1/h) of plane
// p = kbase + PK into the derivative accumulators of output planes
// kbase + s, s = 0..6.
template <int FORM, int PK, class T>
__device__ __forceinline__ void zscatter_d(T (&acc)[7], int kbase, T dv, bool wall, int N) {
  if (!wall) {
#pragma unroll
    for (int s = 0; s < 7; ++s) acc[s] += zdcoef6<FORM, T>(PK - s) * dv;
    return;
  }
#pragma unroll
  for (int s = 0; s < 7; ++s) {
    const int k = kbase + s;
    if (k >= 0 && k < N) acc[s] += zdcoef_wall<FORM, T>(k, kbase + PK, N) * dv;
  }
}

// Tile plane in LDS: (TX + 2H) x (TY + 2H) values of one plane, element
// (x, y) of the tile (x, y may be -H .. T+H-1) at (y + H) * W + (x + H).
template <int TX, int TY, int H> struct Plane {
  static constexpr int W = TX + 2 * H;
  static constexpr int HT = TY + 2 * H;
  static constexpr int N = W * HT;
  static __device__ __forceinline__ int at(int x, int y) { return (y + H) * W + (x + H); }
};

// Cooperative load of plane k of a field into a tile plane buffer.
template <int TX, int TY, int H, class T>
__device__ __forceinline__ void load_plane(T* __restrict__ dst, const T* __restrict__ src,
                                           const BoxDev& b, int x0, int y0, int k) {
  using PL = Plane<TX, TY, H>;
  const long long base = b.off + (long long)k * b.nx * b.ny;
  for (int t = threadIdx.x; t < PL::N; t += TX * TY) {
    const int yy = t / PL::W, xx = t - yy * PL::W;
    const int gx = wrapm(x0 + xx - H, b.nx), gy = wrapm(y0 + yy - H, b.ny);
    dst[t] = src[base + (long long)gy * b.nx + gx];
  }
}

// Items are assigned so that each XCD (blockIdx % 8) works on a contiguous
// range of work items (neighbouring tiles share halo data in that XCD's L2).
__device__ __forceinline__ int xcd_item(int nitems) {
  const int per = (nitems + 7) / 8;
  return (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
}

}  // namespace smhd
