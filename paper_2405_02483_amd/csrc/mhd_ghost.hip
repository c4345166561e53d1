// Closed-wall ghost zones of the z axis (Section 10): one thread per (x, y)
// column position and ghost plane; each launch covers every wall-bounded box
// through a table of (box, cell range) work items.
#include "mhd_kernels.hpp"

namespace smhd {

#define FIELD(name, ptr) \
  auto name = [&](int a, int b, int c) -> T { return ptr[g.at(a, b, c)]; }

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

template <class T>
void launch_ghost(const Launch& L, P8<T> f) {
  if (L.nghost_blk == 0) return;
  const dim3 grid(L.nghost_blk), block(kBlock);
  L.at(PASS_GHOST);
  hipLaunchKernelGGL(k_ghost1<T>, grid, block, 0, L.stream, L.boxes, L.gtab, f);
  hipLaunchKernelGGL(k_ghost2<T>, grid, block, 0, L.stream, L.boxes, L.gtab, f);
  L.at(PASS_END);
}

template void launch_ghost<float>(const Launch&, P8<float>);
template void launch_ghost<double>(const Launch&, P8<double>);

}  // namespace smhd
