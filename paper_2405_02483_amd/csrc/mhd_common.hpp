// Device-side building blocks of the staggered-mesh MHD kernels (gfx950):
// box addressing with periodic wrap, the paper's staggered derivative and
// interpolation operators (Section 4.2 eq. deriv / eq. derivcoef, Section 4.3
// eq. interp / eq. interpcoef), and the reduced-order treatment next to the
// ends of a wall-bounded z axis (Section 10: each operation gives up the
// outermost valid ghost zone).
//
// Storage: arrays are [z][y][x], x fastest.  A face array's element i sits at
// position i - 1/2 (lower index side, Section 4.1).  "dn" operators take
// samples at integer positions to the lower half point of the same index;
// "up" operators take samples at i - 1/2 to position i.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smhd {

enum : unsigned {
  T_CONT = 1u << 0, T_ADV = 1u << 1, T_PRES = 1u << 2, T_VISC = 1u << 3,
  T_LORENTZ = 1u << 4, T_INDUCT = 1u << 5, T_RESIST = 1u << 6,
  T_EDIFF = 1u << 7, T_GRAV = 1u << 8, T_COOL = 1u << 9, T_CORI = 1u << 10,
  T_EDIFFAV = 1u << 11, T_LNP = 1u << 12, T_DIVB = 1u << 13, T_SMAG = 1u << 14,
  T_MAX5 = 1u << 15, T_QUENCH = 1u << 16, T_ORDER2 = 1u << 17
};

constexpr int kBlock = 256;          // threads per workgroup of the cell kernels

// Sixth-order coefficients (eq. derivcoef: 75/64, -25/384, 3/640; eq.
// interpcoef: 150/256, -25/256, 3/256) and the centred 4th-order ones used
// only next to the ends of a wall-bounded axis.
template <class T> struct Cf {
  static constexpr T IA = T(75.0 / 128.0), IB = T(-25.0 / 256.0), IC = T(3.0 / 256.0);
  static constexpr T DA = T(75.0 / 64.0), DB = T(-25.0 / 384.0), DC = T(3.0 / 640.0);
  static constexpr T I4A = T(9.0 / 16.0), I4B = T(-1.0 / 16.0);
  static constexpr T D4A = T(9.0 / 8.0), D4B = T(-1.0 / 24.0);
};

// One box as the kernels see it (lives in device memory, read by every
// thread of a workgroup through the scalar cache).
struct BoxDev {
  int nx, ny, nzt, ngz;      // nzt = nz + 2 ngz planes
  int wall, g0, g1, poff;    // g0 = ngz (first interior plane), g1 = ngz + nz;
                             // poff: first entry of this box in per-plane tables
  long long off;             // first element in the packed field arrays
  long long ncell;           // nx * ny * nzt
  double dx, dy, dz, hmin, hmax;
  long long zoff;            // wall boxes: first entry of the z-coefficient table
  // length factors of the viscosity (eq. nuij): nu_aa = lv[a] <nu>, edge
  // nu_ab = le[ab] <nu> (xy, xz, yz).  Richtmyer-Morton: dx_a and
  // max(dx_a, dx_b); constant viscosity: h_min for all, so that every
  // component is nu_const whatever the cell shape (Section 6.1).
  double lv[3], le[3];
  // per-plane z table (ZJ_COUNT entries per plane) in the z-coefficient
  // array, for every box; stretched: a stretched z axis
  long long joff;
  int stretched;
};

// Per-plane z quantities (Section 4.2: derivatives in index space times the
// Jacobian at the output; uniform boxes hold constants): ZJ_C, ZJ_F the
// Jacobians of up derivatives (outputs at centres) and down derivatives
// (outputs on faces), with the wall end copy built in (the end output no
// stencil reaches takes its neighbour's); ZJ_LZZ nu_zz's length (centre);
// ZJ_LXZ, ZJ_LYZ the y- and x-edge lengths (face heights); ZJ_LZF the
// energy diffusion's z length (faces); ZJ_H the shock and Smagorinsky h;
// ZJ_DZC the centre interval (cell volumes).
enum ZJ : int { ZJ_C = 0, ZJ_F, ZJ_LZZ, ZJ_LXZ, ZJ_LYZ, ZJ_LZF, ZJ_H, ZJ_DZC, ZJ_COUNT };

// z-stencil coefficient tables of wall-bounded boxes: for operator type
// ZT_*, output plane k and offset d = p - k in [-3, 3], the coefficient of
// input plane p (entry (ZT * nzt + k) * 7 + d + 3).  Types: interpolation dn
// / up, derivative dn / up (before 1/h), and the derivative written on first
// differences d_m = f[m] - f[m-1] (dn / up; d = m - k).
enum ZType : int { ZT_IDN = 0, ZT_IUP, ZT_DDN, ZT_DUP, ZT_DDDN, ZT_DDUP, ZT_COUNT };

// Order choice at the ends of a wall-bounded axis of N planes: the widest
// centred stencil (q pairs) around c = k + form whose samples lie in [0, N);
// the one output no stencil reaches takes its neighbour's stencil.
inline void zwall_pairs(int k, int form, int N, int& c, int& q) {
  c = k + form;
  q = c < N - c ? c : N - c;
  if (q > 3) q = 3;
  if (q <= 0) {
    c = form ? N - 1 : 1;
    q = 1;
  }
}

inline double zwall_coef(int type, int k, int p, int N) {
  const int form = (type == ZT_IUP || type == ZT_DUP || type == ZT_DDUP) ? 1 : 0;
  int c, q;
  zwall_pairs(k, form, N, c, q);
  static const double I[4][3] = {{0, 0, 0}, {0.5, 0, 0}, {9.0 / 16.0, -1.0 / 16.0, 0},
                                 {75.0 / 128.0, -25.0 / 256.0, 3.0 / 256.0}};
  static const double D[4][3] = {{0, 0, 0}, {1.0, 0, 0}, {9.0 / 8.0, -1.0 / 24.0, 0},
                                 {75.0 / 64.0, -25.0 / 384.0, 3.0 / 640.0}};
  if (type == ZT_DDDN || type == ZT_DDUP) {
    // weight of the first difference d_p: sum of d_P over pairs P > |p - c|
    const int j = p > c ? p - c : c - p;
    double w = 0.0;
    for (int P = j + 1; P <= q; ++P) w += D[q][P - 1];
    return w;
  }
  const int d = p - c;
  const int P = d >= 0 ? d + 1 : -d;
  if (P > q) return 0.0;
  const bool der = type == ZT_DDN || type == ZT_DUP;
  const double w = der ? D[q][P - 1] : I[q][P - 1];
  return (der && d < 0) ? -w : w;
}

// A workgroup's share of the cells: kBlock consecutive cells of one box.
struct Blk {
  int box;
  int n;                     // valid cells in this block (<= kBlock)
  long long start;           // box-local flat index of the first cell
};

template <class T> struct P8 { T* p[8]; };
template <class T> struct CP8 { const T* p[8]; };

// Box geometry for one thread, with wrapped addressing.  Nested operators
// along one axis never reach further than +-3 cells inside one kernel, and
// every axis has >= 6 cells, so one conditional wrap suffices.
template <class T> struct Geo {
  int nx, ny, nzt, wall, g0, g1;
  long long off, sxy;
  T dx, dy, dz, h, hmax, hxi, hyi, hzi;
  T lx, ly, lz, lxy, lxz, lyz;   // viscosity length factors (BoxDev::lv, le)
  __device__ explicit Geo(const BoxDev& b)
      : nx(b.nx), ny(b.ny), nzt(b.nzt), wall(b.wall), g0(b.g0), g1(b.g1),
        off(b.off), sxy((long long)b.nx * b.ny),
        dx(T(b.dx)), dy(T(b.dy)), dz(T(b.dz)), h(T(b.hmin)), hmax(T(b.hmax)),
        hxi(T(1.0 / b.dx)), hyi(T(1.0 / b.dy)), hzi(T(1.0 / b.dz)),
        lx(T(b.lv[0])), ly(T(b.lv[1])), lz(T(b.lv[2])),
        lxy(T(b.le[0])), lxz(T(b.le[1])), lyz(T(b.le[2])) {}
  __device__ long long at(int i, int j, int k) const {
    i = i < 0 ? i + nx : (i >= nx ? i - nx : i);
    j = j < 0 ? j + ny : (j >= ny ? j - ny : j);
    if (!wall) k = k < 0 ? k + nzt : (k >= nzt ? k - nzt : k);
    return off + (long long)k * sxy + (long long)j * nx + i;
  }
};

// ---------------------------------------------------------------------------
// Pair form of the staggered stencils.  With c the index just above the
// output point (c = i for dn, c = i + 1 for up), pair p is (c+p-1, c-p):
//   interpolation  sum_p w_p (f[c+p-1] + f[c-p])
//   derivative     sum_p d_p (f[c+p-1] - f[c-p]) / h
// FAM: 0 interpolation, 1 derivative.  FORM: 0 dn, 1 up.
template <int FAM, int FORM, class T, class O>
__device__ __forceinline__ T op6(const O& o, T hinv) {
  constexpr int c = FORM;
  const T h1 = o(c), l1 = o(c - 1), h2 = o(c + 1), l2 = o(c - 2), h3 = o(c + 2), l3 = o(c - 3);
  if constexpr (FAM == 0) {
    return Cf<T>::IA * (h1 + l1) + Cf<T>::IB * (h2 + l2) + Cf<T>::IC * (h3 + l3);
  } else {
    return (Cf<T>::DA * (h1 - l1) + Cf<T>::DB * (h2 - l2) + Cf<T>::DC * (h3 - l3)) * hinv;
  }
}

// Wall-bounded z: the widest centred stencil (q pairs, q = 3, 2, 1) whose
// samples lie inside [0, N); the one output no stencil reaches (dn at k = 0,
// up at k = N-1) takes its neighbour's value.  `f(kk)` returns plane kk.
template <int FAM, int FORM, class T, class F>
__device__ __forceinline__ T opwall(const F& f, int k, int N, T hinv) {
  int c = k + FORM;
  int q = min(3, min(c, N - c));
  if (q == 0) { c = FORM ? N - 1 : 1; q = 1; }
  if (q == 3) {
    return op6<FAM, FORM, T>([&](int m) { return f(c - FORM + m); }, hinv);
  }
  if (q == 2) {
    const T h1 = f(c), l1 = f(c - 1), h2 = f(c + 1), l2 = f(c - 2);
    if constexpr (FAM == 0) return Cf<T>::I4A * (h1 + l1) + Cf<T>::I4B * (h2 + l2);
    else return (Cf<T>::D4A * (h1 - l1) + Cf<T>::D4B * (h2 - l2)) * hinv;
  }
  const T h1 = f(c), l1 = f(c - 1);
  if constexpr (FAM == 0) return T(0.5) * (h1 + l1);
  else return (h1 - l1) * hinv;
}

// Named operators on a point functor F(i, j, k).
template <class T, class F> __device__ __forceinline__ T Xdn(const Geo<T>&, const F& f, int i, int j, int k) {
  return op6<0, 0, T>([&](int m) { return f(i + m, j, k); }, T(0));
}
template <class T, class F> __device__ __forceinline__ T Xup(const Geo<T>&, const F& f, int i, int j, int k) {
  return op6<0, 1, T>([&](int m) { return f(i + m, j, k); }, T(0));
}
template <class T, class F> __device__ __forceinline__ T DXdn(const Geo<T>& g, const F& f, int i, int j, int k) {
  return op6<1, 0, T>([&](int m) { return f(i + m, j, k); }, g.hxi);
}
template <class T, class F> __device__ __forceinline__ T DXup(const Geo<T>& g, const F& f, int i, int j, int k) {
  return op6<1, 1, T>([&](int m) { return f(i + m, j, k); }, g.hxi);
}
template <class T, class F> __device__ __forceinline__ T Ydn(const Geo<T>&, const F& f, int i, int j, int k) {
  return op6<0, 0, T>([&](int m) { return f(i, j + m, k); }, T(0));
}
template <class T, class F> __device__ __forceinline__ T Yup(const Geo<T>&, const F& f, int i, int j, int k) {
  return op6<0, 1, T>([&](int m) { return f(i, j + m, k); }, T(0));
}
template <class T, class F> __device__ __forceinline__ T DYdn(const Geo<T>& g, const F& f, int i, int j, int k) {
  return op6<1, 0, T>([&](int m) { return f(i, j + m, k); }, g.hyi);
}
template <class T, class F> __device__ __forceinline__ T DYup(const Geo<T>& g, const F& f, int i, int j, int k) {
  return op6<1, 1, T>([&](int m) { return f(i, j + m, k); }, g.hyi);
}
template <int FAM, int FORM, class T, class F>
__device__ __forceinline__ T zop(const Geo<T>& g, const F& f, int i, int j, int k, T hinv) {
  if (g.wall) return opwall<FAM, FORM, T>([&](int kk) { return f(i, j, kk); }, k, g.nzt, hinv);
  return op6<FAM, FORM, T>([&](int m) { return f(i, j, k + m); }, hinv);
}
template <class T, class F> __device__ __forceinline__ T Zdn(const Geo<T>& g, const F& f, int i, int j, int k) {
  return zop<0, 0, T>(g, f, i, j, k, T(0));
}
template <class T, class F> __device__ __forceinline__ T Zup(const Geo<T>& g, const F& f, int i, int j, int k) {
  return zop<0, 1, T>(g, f, i, j, k, T(0));
}
template <class T, class F> __device__ __forceinline__ T DZdn(const Geo<T>& g, const F& f, int i, int j, int k) {
  return zop<1, 0, T>(g, f, i, j, k, g.hzi);
}
template <class T, class F> __device__ __forceinline__ T DZup(const Geo<T>& g, const F& f, int i, int j, int k) {
  return zop<1, 1, T>(g, f, i, j, k, g.hzi);
}

template <class T> __device__ __forceinline__ T norm3(T a, T b, T c) {
  T s = a * a + b * b + c * c;
  return s > T(0) ? sqrt(s) : T(0);
}

// Decode this thread's cell; returns false for the idle tail of a block.
struct CellIdx { int box, i, j, k; };
__device__ __forceinline__ bool cell_of(const BoxDev* boxes, const Blk* tab, CellIdx& c,
                                        BoxDev& b) {
  const Blk t = tab[blockIdx.x];
  if ((int)threadIdx.x >= t.n) return false;
  b = boxes[t.box];
  // boxes hold fewer than 2^31 cells (checked by mhd_init): 32-bit division
  unsigned q = (unsigned)t.start + threadIdx.x;
  const unsigned nx = (unsigned)b.nx, ny = (unsigned)b.ny;
  c.box = t.box;
  const unsigned qx = q / nx;
  c.i = (int)(q - qx * nx);
  const unsigned qy = qx / ny;
  c.j = (int)(qx - qy * ny);
  c.k = (int)qy;
  return true;
}

}  // namespace smhd
