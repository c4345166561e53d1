// Float64 reductions over the interior cells: conserved totals, div B norms,
// maximum signal / diffusion / rate speeds for the Courant condition (eq.
// courantcond) with the cell that attains them, and non-finite / non-positive
// counts.  Two deterministic passes: a fixed-shape tree per workgroup writes
// one partial record per work item; one workgroup then folds the partials in
// a fixed order.  No atomics, so repeated calls give identical bits.  Ties in
// a maximum resolve to the smallest packed cell index.
#include "mhd_kernels.hpp"

namespace smhd {

__device__ __forceinline__ double bsum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ void bmaxarg(double& v, long long& a, double* sh, long long* sa) {
  const int t = threadIdx.x;
  sh[t] = v;
  sa[t] = a;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (t < s) {
      const double o = sh[t + s];
      const long long oa = sa[t + s];
      if (o > sh[t] || (o == sh[t] && oa < sa[t])) {
        sh[t] = o;
        sa[t] = oa;
      }
    }
    __syncthreads();
  }
  v = sh[0];
  a = sa[0];
  __syncthreads();
}

__device__ __forceinline__ long long bcount(long long v, long long* sa) {
  const int t = threadIdx.x;
  sa[t] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (t < s) sa[t] += sa[t + s];
    __syncthreads();
  }
  const long long r = sa[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ bool finite_d(double x) { return x == x && fabs(x) <= 1.79e308; }

template <class T>
__global__ __launch_bounds__(kBlock) void k_reduce(const BoxDev* boxes, const Blk* tab, CP8<T> f,
                                                   CP8<T> dfdt, const T* __restrict__ ux,
                                                   const T* __restrict__ uy,
                                                   const T* __restrict__ uz,
                                                   const T* __restrict__ nt, Phys<T> ph,
                                                   RedPartial* __restrict__ part) {
  __shared__ double sh[kBlock];
  __shared__ long long sa[kBlock];
  double s[kNSum];
  double mx[kNMax];
  long long arg[kNArg];
  long long nonfin = 0, nonpos = 0;
  for (int q = 0; q < kNSum; ++q) s[q] = 0.0;
  for (int q = 0; q < kNMax; ++q) mx[q] = 0.0;
  for (int q = 0; q < kNArg; ++q) arg[q] = 0x7fffffffffffffffLL;

  const Blk t = tab[blockIdx.x];
  if ((int)threadIdx.x < t.n) {
    const BoxDev b = boxes[t.box];
    const Geo<T> g(b);
    long long q = t.start + threadIdx.x;
    const int i = (int)(q % b.nx);
    q /= b.nx;
    const int j = (int)(q % b.ny);
    const int k = (int)(q / b.ny);
    const bool interior = !b.wall || (k >= b.g0 && k < b.g1);
    if (interior) {
      const long long o = g.at(i, j, k);
      auto R = [&](int x_, int y_, int z_) -> T { return f.p[0][g.at(x_, y_, z_)]; };
      auto BX = [&](int x_, int y_, int z_) -> T { return f.p[5][g.at(x_, y_, z_)]; };
      auto BY = [&](int x_, int y_, int z_) -> T { return f.p[6][g.at(x_, y_, z_)]; };
      auto BZ = [&](int x_, int y_, int z_) -> T { return f.p[7][g.at(x_, y_, z_)]; };
      auto UX = [&](int x_, int y_, int z_) -> T { return ux[g.at(x_, y_, z_)]; };
      auto UY = [&](int x_, int y_, int z_) -> T { return uy[g.at(x_, y_, z_)]; };
      auto UZ = [&](int x_, int y_, int z_) -> T { return uz[g.at(x_, y_, z_)]; };
      const double r = f.p[0][o], px = f.p[1][o], py = f.p[2][o], pz = f.p[3][o];
      const double e = f.p[4][o], bx = f.p[5][o], by = f.p[6][o], bz = f.p[7][o];
      for (int v = 0; v < 8; ++v)
        if (!finite_d((double)f.p[v][o])) ++nonfin;
      if (!(r > 0.0) || !(e > 0.0)) ++nonpos;
      const double rx = Xdn(g, R, i, j, k), ry = Ydn(g, R, i, j, k), rz = Zdn(g, R, i, j, k);
      const double dV = b.dx * b.dy * b.dz;    // totals are volume integrals
      s[0] = r * dV;
      s[1] = px * dV;
      s[2] = py * dV;
      s[3] = pz * dV;
      s[4] = (0.5 * px * px / rx + 0.5 * py * py / ry + 0.5 * pz * pz / rz) * dV;
      s[5] = (bx * bx + by * by + bz * bz) * dV;
      s[6] = e * dV;
      const double divb = (double)DXup(g, BX, i, j, k) + (double)DYup(g, BY, i, j, k) +
                          (double)DZup(g, BZ, i, j, k);
      s[7] = divb * divb;
      mx[0] = fabs(divb);
      mx[1] = fmax(fabs(bx), fmax(fabs(by), fabs(bz)));
      mx[2] = fmax(fabs((double)ux[o]), fmax(fabs((double)uy[o]), fabs((double)uz[o])));
      // signal speed c_s + c_A + |u perpendicular to B| at the centre
      const double ubx = Xup(g, UX, i, j, k), uby = Yup(g, UY, i, j, k), ubz = Zup(g, UZ, i, j, k);
      const double bbx = Xup(g, BX, i, j, k), bby = Yup(g, BY, i, j, k), bbz = Zup(g, BZ, i, j, k);
      const double P = (double)ph.gamma1 * e;
      const double cs = sqrt((double)ph.gamma * P / r);
      const double bb = sqrt(bbx * bbx + bby * bby + bbz * bbz);
      const double ca = bb / sqrt((double)ph.mu * r);
      const double udotb = bb > 0.0 ? (ubx * bbx + uby * bby + ubz * bbz) / bb : 0.0;
      const double uu = ubx * ubx + uby * uby + ubz * ubz;
      const double up = sqrt(fmax(uu - udotb * udotb, 0.0));
      const long long packed = b.off + ((long long)k * b.ny + j) * b.nx + i;
      mx[3] = cs + ca + up;
      arg[0] = packed;
      const double nu = nt[o];
      const double eta_speed =
          (double)ph.eta_const > 0.0 ? (double)ph.eta_const / b.hmin : (double)ph.nuB * nu;
      mx[4] = fmax(nu, eta_speed * (b.hmax / b.hmin));
      arg[1] = packed;
      if (dfdt.p[0]) {
        const double dr = (double)dfdt.p[0][o] / r;
        const double dem = (double)dfdt.p[4][o] / e - dr;
        mx[5] = fmax(fabs(dr), fabs(dem));
        arg[2] = packed;
      }
    }
  }
  RedPartial* out = part + blockIdx.x;
  for (int q = 0; q < kNSum; ++q) {
    const double v = bsum(s[q], sh);
    if (threadIdx.x == 0) out->sum[q] = v;
  }
  for (int q = 0; q < 3; ++q) {
    double v = mx[q];
    long long a = 0;
    bmaxarg(v, a, sh, sa);
    if (threadIdx.x == 0) out->mx[q] = v;
  }
  for (int q = 3; q < 6; ++q) {
    double v = mx[q];
    long long a = arg[q - 3];
    bmaxarg(v, a, sh, sa);
    if (threadIdx.x == 0) {
      out->mx[q] = v;
      out->arg[q - 3] = a;
    }
  }
  const long long c1 = bcount(nonfin, sa);
  const long long c2 = bcount(nonpos, sa);
  if (threadIdx.x == 0) {
    out->mx[6] = 0.0;
    out->nonfinite = c1;
    out->nonpositive = c2;
  }
}

__global__ __launch_bounds__(kBlock) void k_reduce_final(const RedPartial* __restrict__ part,
                                                         int n, RedPartial* __restrict__ tot) {
  __shared__ double sh[kBlock];
  __shared__ long long sa[kBlock];
  double s[kNSum];
  double mx[kNMax];
  long long arg[kNArg];
  long long c1 = 0, c2 = 0;
  for (int q = 0; q < kNSum; ++q) s[q] = 0.0;
  for (int q = 0; q < kNMax; ++q) mx[q] = 0.0;
  for (int q = 0; q < kNArg; ++q) arg[q] = 0x7fffffffffffffffLL;
  for (int p = threadIdx.x; p < n; p += kBlock) {
    const RedPartial& r = part[p];
    for (int q = 0; q < kNSum; ++q) s[q] += r.sum[q];
    for (int q = 0; q < 3; ++q) mx[q] = fmax(mx[q], r.mx[q]);
    for (int q = 3; q < 6; ++q) {
      const double v = r.mx[q];
      const long long a = r.arg[q - 3];
      if (v > mx[q] || (v == mx[q] && a < arg[q - 3])) {
        mx[q] = v;
        arg[q - 3] = a;
      }
    }
    c1 += r.nonfinite;
    c2 += r.nonpositive;
  }
  for (int q = 0; q < kNSum; ++q) {
    const double v = bsum(s[q], sh);
    if (threadIdx.x == 0) tot->sum[q] = v;
  }
  for (int q = 0; q < 3; ++q) {
    double v = mx[q];
    long long a = 0;
    bmaxarg(v, a, sh, sa);
    if (threadIdx.x == 0) tot->mx[q] = v;
  }
  for (int q = 3; q < 6; ++q) {
    double v = mx[q];
    long long a = arg[q - 3];
    bmaxarg(v, a, sh, sa);
    if (threadIdx.x == 0) {
      tot->mx[q] = v;
      tot->arg[q - 3] = a;
    }
  }
  const long long t1 = bcount(c1, sa);
  const long long t2 = bcount(c2, sa);
  if (threadIdx.x == 0) {
    tot->mx[6] = 0.0;
    tot->nonfinite = t1;
    tot->nonpositive = t2;
  }
}

template <class T>
void launch_reduce(const Launch& L, CP8<T> f, CP8<T> dfdt, const Work<T>& w, const Phys<T>& ph,
                   RedPartial* partial, RedPartial* total) {
  hipLaunchKernelGGL(k_reduce<T>, dim3(L.nblk), dim3(kBlock), 0, L.stream, L.boxes, L.tab, f,
                     dfdt, w.ux, w.uy, w.uz, w.nt, ph, partial);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, L.stream, partial, L.nblk, total);
}

template void launch_reduce<float>(const Launch&, CP8<float>, CP8<float>, const Work<float>&,
                                   const Phys<float>&, RedPartial*, RedPartial*);
template void launch_reduce<double>(const Launch&, CP8<double>, CP8<double>, const Work<double>&,
                                    const Phys<double>&, RedPartial*, RedPartial*);

}  // namespace smhd
