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

// Per-item partial results of the float64 reductions (mhd_reductions),
// written by the reduction instantiations of passes A1 (everything but the
// diffusion speed) and A2 (the diffusion speed).  Sums are over the item's
// interior cells; the first seven are weighted by the cell volume.
struct RedItem {
  double sum[8];        // mass, px, py, pz, ekin, B^2, e, (div B)^2 (unweighted)
  double mx[3];         // max |div B|, max |B_a|, max |u_a|
  double cmax, dmax, rmax;          // wave speed, diffusion speed, rate
  long long carg, darg, rarg;       // their cells (packed index, first maximal)
  long long nonfinite, nonpositive;
};

// Totals of all items and the three Courant limits (eq. courantcond), each
// from its box's own spacing, with the cell that sets each.
struct RedTotal {
  double sum[8];
  double mx[3];
  double cmax, dmax, rmax;
  double dtw, dtd, dtr;
  long long warg, darg, rarg;
  long long nonfinite, nonpositive;
};

// Wavefront reductions (64 lanes): the result is exact in lane 0; every lane
// combines in a fixed order, so the result does not depend on timing.
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ long long wave_isum(long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// (max, first index): ties go to the smaller index
__device__ __forceinline__ void wave_maxarg(double& v, long long& a) {
  for (int o = 32; o > 0; o >>= 1) {
    const double v2 = __shfl_xor(v, o, 64);
    const long long a2 = __shfl_xor(a, o, 64);
    if (v2 > v || (v2 == v && a2 < a)) {
      v = v2;
      a = a2;
    }
  }
}

__device__ __forceinline__ int wrapm(int a, int n) {
  const int r = a % n;
  return r < 0 ? r + n : r;
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
// plane q.  Periodic boxes, and planes whose full stencil lies inside a
// wall-bounded box: the sixth-order stencil on differences; planes next to a
// wall end: the box's coefficient table zt (type ZT), read through the
// scalar cache.  FAM 0 interpolation, 1 derivative; FORM 0 dn, 1 up.
template <int FAM, int FORM, int W, int LAG, class T>
__device__ __forceinline__ T zwin(const T (&w)[W], int q, bool wall, int N, T hinv,
                                  const T* __restrict__ zt) {
  static_assert(LAG >= 3 - FORM && W - 1 - LAG >= 2 + FORM, "window too short");
  if (!wall || (q >= 3 && q <= N - 4)) {
    return op6<FAM, FORM, T>([&](int m) { return w[LAG + m]; }, hinv);
  }
  constexpr int type = FAM == 0 ? (FORM ? ZT_IUP : ZT_IDN) : (FORM ? ZT_DUP : ZT_DDN);
  const T* c = zt + ((long long)type * N + q) * 7 + 3 - LAG;   // c[m]: slot m
  T acc = T(0);
#pragma unroll
  for (int m = (LAG - 3 > 0 ? LAG - 3 : 0); m < (LAG + 4 < W ? LAG + 4 : W); ++m) acc += c[m] * w[m];
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
__device__ __forceinline__ void zscatter(T (&acc)[7], int kbase, T v, bool wall, int N,
                                         const T* __restrict__ zt) {
  if (!wall || (kbase >= 3 && kbase + 6 <= N - 4)) {
#pragma unroll
    for (int s = 0; s < 7; ++s) acc[s] += zcoef6<FAM, FORM, T>(PK - s) * v;
    return;
  }
  constexpr int type = FAM == 0 ? (FORM ? ZT_IUP : ZT_IDN) : (FORM ? ZT_DUP : ZT_DDN);
#pragma unroll
  for (int s = 0; s < 7; ++s) {
    const int k = kbase + s;
    if (k >= 0 && k < N) acc[s] += zt[((long long)type * N + k) * 7 + PK - s + 3] * v;
  }
}

// Staggered derivative written on first differences d_m = f[m] - f[m-1]:
// with c = k + FORM and q pairs, f[c+P-1] - f[c-P] telescopes into the sum
// of d_m over |m - c| <= P - 1, so output k = sum_m W(k, m) d_m / h with
// W = sum of the pair coefficients d_P over P > |m - c|.  Scattering d_m
// (instead of f) keeps the rounding relative to the differences, as in the
// gather form, where a plain scatter of f would round relative to |f|.
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
__device__ __forceinline__ void zscatter_d(T (&acc)[7], int kbase, T dv, bool wall, int N,
                                           const T* __restrict__ zt) {
  if (!wall || (kbase >= 3 && kbase + 6 <= N - 4)) {
#pragma unroll
    for (int s = 0; s < 7; ++s) acc[s] += zdcoef6<FORM, T>(PK - s) * dv;
    return;
  }
  constexpr int type = FORM ? ZT_DDUP : ZT_DDDN;
#pragma unroll
  for (int s = 0; s < 7; ++s) {
    const int k = kbase + s;
    if (k >= 0 && k < N) acc[s] += zt[((long long)type * N + k) * 7 + PK - s + 3] * dv;
  }
}

// The same on a stretched z axis: dv without the 1/h, each output plane's
// share times that plane's Jacobian js[s] (derivatives in index space times
// the Jacobian at the output).
template <int FORM, int PK, class T>
__device__ __forceinline__ void zscatter_dj(T (&acc)[7], int kbase, T dv, const T (&js)[7], bool wall, int N,
                                            const T* __restrict__ zt) {
  if (!wall || (kbase >= 3 && kbase + 6 <= N - 4)) {
#pragma unroll
    for (int s = 0; s < 7; ++s) acc[s] += zdcoef6<FORM, T>(PK - s) * dv * js[s];
    return;
  }
  constexpr int type = FORM ? ZT_DDUP : ZT_DDDN;
#pragma unroll
  for (int s = 0; s < 7; ++s) {
    const int k = kbase + s;
    if (k >= 0 && k < N) acc[s] += zt[((long long)type * N + k) * 7 + PK - s + 3] * dv * js[s];
  }
}

// Tile plane in LDS: (TX + 2HX) x (TY + 2HY) values of one plane, element
// (x, y) of the tile (x in -HX .. TX+HX-1, y in -HY .. TY+HY-1) at
// (y + HY) * W + (x + HX).
template <int TX, int TY, int HX, int HY = HX> struct Plane {
  static constexpr int W = TX + 2 * HX;
  static constexpr int HT = TY + 2 * HY;
  static constexpr int N = W * HT;
  // buffer size: N rounded up to whole passes of the workgroup, so that the
  // cooperative loads need no bounds test (see load_plane)
  static constexpr int NP = (N + TX * TY - 1) / (TX * TY) * (TX * TY);
  static __device__ __forceinline__ int at(int x, int y) { return (y + HY) * W + (x + HX); }
};

// In-plane offsets (periodic wrap in x and y already applied) of the tile
// plane elements this thread loads: element t = threadIdx.x + i * (TX*TY).
// They do not change from plane to plane, so they are computed once.
template <int TX, int TY, int HX, int HY = HX> struct PlaneIdx {
  using PL = Plane<TX, TY, HX, HY>;
  static constexpr int NT = TX * TY;
  static constexpr int NPER = (PL::N + NT - 1) / NT;
  int off[NPER];
  __device__ __forceinline__ void init(const BoxDev& b, int x0, int y0) {
#pragma unroll
    for (int i = 0; i < NPER; ++i) {
      const int t = (int)threadIdx.x + i * NT;
      const int yy = t / PL::W, xx = t - yy * PL::W;
      off[i] = t < PL::N ? wrapm(y0 + yy - HY, b.ny) * b.nx + wrapm(x0 + xx - HX, b.nx) : 0;
    }
  }
};

// Cooperative load of plane k of a field into a tile plane buffer of
// Plane::NP elements.  Slots past N load element 0 of the plane (offset 0)
// into the padding: no bounds test, so no branch separates a load from its
// store, and the loads of several planes can all be in flight at once.
template <int TX, int TY, int HX, int HY, class T>
__device__ __forceinline__ void load_plane(T* __restrict__ dst, const T* __restrict__ src,
                                           const BoxDev& b, const PlaneIdx<TX, TY, HX, HY>& ix,
                                           int k) {
  using PX = PlaneIdx<TX, TY, HX, HY>;
  static_assert(PX::NPER * PX::NT == PX::PL::NP, "plane padding");
  const T* __restrict__ s = src + b.off + (long long)k * b.nx * b.ny;
#pragma unroll
  for (int i = 0; i < PX::NPER; ++i) dst[(int)threadIdx.x + i * PX::NT] = s[ix.off[i]];
}

// Items are assigned so that each XCD (blockIdx % 8) works on a contiguous
// range of work items (neighbouring tiles share halo data in that XCD's L2).
__device__ __forceinline__ int xcd_item(int nitems) {
  const int per = (nitems + 7) / 8;
  return (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
}

// Persistent mode: the next item for this workgroup, from the range of its
// own XCD first (workgroups are dispatched to the 8 XCDs round-robin, so
// blockIdx % 8 is the XCD), then from the other ranges in turn.  queue[x]
// counts the items of range x handed out; nitems when everything is taken.
__device__ __forceinline__ int zpull(int nitems, int* queue) {
  const int per = (nitems + 7) / 8;
  const int x0 = (int)(blockIdx.x % 8);
  for (int d = 0; d < 8; ++d) {
    const int x = (x0 + d) % 8;
    const int lo = x * per;
    const int cnt = min(per, nitems - lo);
    if (cnt <= 0) continue;
    if (__hip_atomic_load(&queue[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= cnt) continue;
    const int t = atomicAdd(&queue[x], 1);
    if (t < cnt) return lo + t;
  }
  return nitems;
}

// First and next item of a workgroup (all threads call; thread 0 pulls and
// broadcasts through LDS).  Grid mode (PERS false): one item each.
template <bool PERS>
__device__ __forceinline__ int zfirst(int nitems, int* queue, int* s) {
  if constexpr (!PERS) return xcd_item(nitems);
  if (threadIdx.x == 0) *s = zpull(nitems, queue);
  __syncthreads();
  return *s;
}

template <bool PERS>
__device__ __forceinline__ int znext(int nitems, int* queue, int* s) {
  if constexpr (!PERS) return nitems;
  __syncthreads();
  if (threadIdx.x == 0) *s = zpull(nitems, queue);
  __syncthreads();
  return *s;
}

}  // namespace smhd
