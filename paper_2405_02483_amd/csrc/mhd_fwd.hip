// Cell-parallel kernels outside the stage path: the viscosity chain used by
// the float64 reductions (face velocities, speed-like viscosity nu1|u| +
// nu3(c_s + c_A) + nu2 h max(0, -div u) (eq. RMnu), maximum over the 3x3x3
// neighbourhood and three-cell means (Section 6.1.1)), and the closed-wall
// ghost-zone fill (Section 10).  One thread per cell; each launch covers
// every box through a table of (box, cell range) work items.
#include "mhd_kernels.hpp"

namespace smhd {

#define CELL_PROLOGUE                                   \
  CellIdx ci;                                           \
  BoxDev bx_;                                           \
  if (!cell_of(boxes, tab, ci, bx_)) return;            \
  const Geo<T> g(bx_);                                  \
  const int i = ci.i, j = ci.j, k = ci.k;               \
  const long long o = g.at(i, j, k);

#define FIELD(name, ptr) \
  auto name = [&](int a, int b, int c) -> T { return ptr[g.at(a, b, c)]; }

template <class T>
__global__ __launch_bounds__(kBlock) void k_prim(const BoxDev* boxes, const Blk* tab, CP8<T> f,
                                                 T* __restrict__ ux, T* __restrict__ uy,
                                                 T* __restrict__ uz) {
  CELL_PROLOGUE
  const T* __restrict__ rho = f.p[0];
  FIELD(R, rho);
  ux[o] = f.p[1][o] / Xdn(g, R, i, j, k);
  uy[o] = f.p[2][o] / Ydn(g, R, i, j, k);
  uz[o] = f.p[3][o] / Zdn(g, R, i, j, k);
}

template <class T>
__device__ __forceinline__ void centre_speeds(const Geo<T>& g, const Phys<T>& ph, const T* rho,
                                              const T* e, const T* bxp, const T* byp,
                                              const T* bzp, const T* ux, const T* uy,
                                              const T* uz, int i, int j, int k, T& ubx, T& uby,
                                              T& ubz, T& bbx, T& bby, T& bbz, T& D, T& cs,
                                              T& ca) {
  FIELD(UX, ux);
  FIELD(UY, uy);
  FIELD(UZ, uz);
  FIELD(BX, bxp);
  FIELD(BY, byp);
  FIELD(BZ, bzp);
  const long long o = g.at(i, j, k);
  ubx = Xup(g, UX, i, j, k);
  uby = Yup(g, UY, i, j, k);
  ubz = Zup(g, UZ, i, j, k);
  bbx = Xup(g, BX, i, j, k);
  bby = Yup(g, BY, i, j, k);
  bbz = Zup(g, BZ, i, j, k);
  D = DXup(g, UX, i, j, k) + DYup(g, UY, i, j, k) + DZup(g, UZ, i, j, k);
  const T r = rho[o];
  const T P = ph.gamma1 * e[o];
  cs = sqrt(ph.gamma * P / r);
  ca = norm3(bbx, bby, bbz) / sqrt(ph.mu * r);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_nus(const BoxDev* boxes, const Blk* tab, CP8<T> f,
                                                const T* __restrict__ ux,
                                                const T* __restrict__ uy,
                                                const T* __restrict__ uz, Phys<T> ph,
                                                T* __restrict__ nus) {
  CELL_PROLOGUE
  if (ph.nu_const > T(0)) {
    nus[o] = ph.nu_const / g.h;
    return;
  }
  T ubx, uby, ubz, bbx, bby, bbz, D, cs, ca;
  centre_speeds(g, ph, f.p[0], f.p[4], f.p[5], f.p[6], f.p[7], ux, uy, uz, i, j, k, ubx, uby,
                ubz, bbx, bby, bbz, D, cs, ca);
  const T relu = -D > T(0) ? -D : T(0);
  nus[o] = ph.nu1 * norm3(ubx, uby, ubz) + ph.nu3 * (cs + ca) + ph.nu2 * g.h * relu;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_max3(const BoxDev* boxes, const Blk* tab,
                                                 const T* __restrict__ src,
                                                 T* __restrict__ dst) {
  CELL_PROLOGUE
  T m = src[o];
  for (int dz = -1; dz <= 1; ++dz) {
    const int kk = k + dz;
    if (g.wall && (kk < 0 || kk >= g.nzt)) continue;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) m = fmax(m, src[g.at(i + dx, j + dy, kk)]);
  }
  dst[o] = m;
}

// Three-cell means along x, then y, then z (over the available planes at the
// ends of a wall-bounded z axis), the floor, and ln of the result.
template <class T>
__global__ __launch_bounds__(kBlock) void k_mean3(const BoxDev* boxes, const Blk* tab,
                                                  const T* __restrict__ m, T* __restrict__ nt,
                                                  T* __restrict__ lnt) {
  CELL_PROLOGUE
  T sz = T(0);
  int cnt = 0;
  for (int dz = -1; dz <= 1; ++dz) {
    const int kk = k + dz;
    if (g.wall && (kk < 0 || kk >= g.nzt)) continue;
    T sy = T(0);
    for (int dy = -1; dy <= 1; ++dy) {
      const T sx = (m[g.at(i - 1, j + dy, kk)] + m[g.at(i, j + dy, kk)] +
                    m[g.at(i + 1, j + dy, kk)]) / T(3);
      sy = dy == -1 ? sx : sy + sx;
    }
    sy = sy / T(3);
    sz = cnt == 0 ? sy : sz + sy;
    ++cnt;
  }
  T v = sz / T(cnt);
  v = v > T(1e-30) ? v : T(1e-30);
  nt[o] = v;
  lnt[o] = log(v);
}

// ---------------------------------------------------------------------------
// Closed-wall ghost zones (Section 10 "Closed").  Pass 1: density and energy
// (ln rho and ln e_m extrapolated linearly from the two nearest interior
// cells), parallel field antisymmetric, normal mass flux antisymmetric and
// zero on the wall faces, normal field symmetric.  Pass 2 (needs the new
// ghost density): parallel velocities symmetric.  One thread per (x, y)
// column position and ghost plane.
template <class T>
__global__ __launch_bounds__(kBlock) void k_ghost1(const BoxDev* boxes, const Blk* gtab, P8<T> f) {
  const Blk t = gtab[blockIdx.x];
  if ((int)threadIdx.x >= t.n) return;
  const BoxDev b = boxes[t.box];
  const Geo<T> g(b);
  long long q = t.start + threadIdx.x;      // over nx*ny*(2*ngz)
  const int i = (int)(q % b.nx);
  q /= b.nx;
  const int j = (int)(q % b.ny);
  const int s = (int)(q / b.ny);            // 0 .. 2*ngz-1
  const int g0 = b.g0, g1 = b.g1, N = b.nzt;
  const bool lower = s < b.ngz;
  const int k = lower ? s : g1 + (s - b.ngz);
  T* rho = f.p[0];
  T* e = f.p[4];
  const int a0 = lower ? g0 : g1 - 1, a1 = lower ? g0 + 1 : g1 - 2;
  const T d = T(lower ? g0 - k : k - g1 + 1);
  const T r0 = rho[g.at(i, j, a0)], r1 = rho[g.at(i, j, a1)];
  const T lr0 = log(r0), lr1 = log(r1);
  const T lm0 = log(e[g.at(i, j, a0)] / r0), lm1 = log(e[g.at(i, j, a1)] / r1);
  const T rn = exp(lr0 + d * (lr0 - lr1));
  const long long o = g.at(i, j, k);
  rho[o] = rn;
  e[o] = rn * exp(lm0 + d * (lm0 - lm1));
  const int m = lower ? 2 * g0 - 1 - k : 2 * g1 - 1 - k;
  f.p[5][o] = -f.p[5][g.at(i, j, m)];
  f.p[6][o] = -f.p[6][g.at(i, j, m)];
  // z-faces: wall face itself (pz = 0) and the faces beyond it
  if (lower) {
    const int mf = 2 * g0 - k;
    f.p[3][o] = -f.p[3][g.at(i, j, mf)];
    f.p[7][o] = f.p[7][g.at(i, j, mf)];
    if (s == b.ngz - 1) f.p[3][g.at(i, j, g0)] = T(0);
  } else {
    if (k == g1) {
      f.p[3][o] = T(0);
    } else {
      const int mf = 2 * g1 - k;
      f.p[3][o] = -f.p[3][g.at(i, j, mf)];
      f.p[7][o] = f.p[7][g.at(i, j, mf)];
    }
  }
  (void)N;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_ghost2(const BoxDev* boxes, const Blk* gtab, P8<T> f) {
  const Blk t = gtab[blockIdx.x];
  if ((int)threadIdx.x >= t.n) return;
  const BoxDev b = boxes[t.box];
  const Geo<T> g(b);
  long long q = t.start + threadIdx.x;
  const int i = (int)(q % b.nx);
  q /= b.nx;
  const int j = (int)(q % b.ny);
  const int s = (int)(q / b.ny);
  const bool lower = s < b.ngz;
  const int k = lower ? s : b.g1 + (s - b.ngz);
  const int m = lower ? 2 * b.g0 - 1 - k : 2 * b.g1 - 1 - k;
  const T* rho = f.p[0];
  FIELD(R, rho);
  const long long o = g.at(i, j, k), om = g.at(i, j, m);
  f.p[1][o] = Xdn(g, R, i, j, k) * (f.p[1][om] / Xdn(g, R, i, j, m));
  f.p[2][o] = Ydn(g, R, i, j, k) * (f.p[2][om] / Ydn(g, R, i, j, m));
}

// ---------------------------------------------------------------------------
// Launchers.
// The viscosity chain alone (for the float64 reductions; timed as part of
// the reduction pass by the caller).
template <class T>
void launch_nu(const Launch& L, CP8<T> f, const Work<T>& w, const Phys<T>& ph) {
  const dim3 grid(L.nblk), block(kBlock);
  hipLaunchKernelGGL(k_prim<T>, grid, block, 0, L.stream, L.boxes, L.tab, f, w.ux, w.uy, w.uz);
  hipLaunchKernelGGL(k_nus<T>, grid, block, 0, L.stream, L.boxes, L.tab, f, w.ux, w.uy, w.uz,
                     ph, w.nus);
  hipLaunchKernelGGL(k_max3<T>, grid, block, 0, L.stream, L.boxes, L.tab, w.nus, w.nmax);
  hipLaunchKernelGGL(k_mean3<T>, grid, block, 0, L.stream, L.boxes, L.tab, w.nmax, w.nt, w.lnt);
}

template <class T>
void launch_ghost(const Launch& L, P8<T> f) {
  if (L.nghost_blk == 0) return;
  const dim3 grid(L.nghost_blk), block(kBlock);
  L.at(PASS_GHOST);
  hipLaunchKernelGGL(k_ghost1<T>, grid, block, 0, L.stream, L.boxes, L.gtab, f);
  hipLaunchKernelGGL(k_ghost2<T>, grid, block, 0, L.stream, L.boxes, L.gtab, f);
  L.at(PASS_END);
}

template void launch_nu<float>(const Launch&, CP8<float>, const Work<float>&, const Phys<float>&);
template void launch_nu<double>(const Launch&, CP8<double>, const Work<double>&, const Phys<double>&);
template void launch_ghost<float>(const Launch&, P8<float>);
template void launch_ghost<double>(const Launch&, P8<double>);

}  // namespace smhd
