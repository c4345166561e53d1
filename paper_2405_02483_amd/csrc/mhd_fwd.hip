// Forward kernels of the staggered MHD right-hand side and the RK3 stage.
//
// One RK stage runs these passes over all cells of all boxes (each pass is a
// single launch over a table of (box, cell range) work items):
//   prim    u_a = p_a / adn(rho)                              (Section 4.1)
//   nus     speed-like viscosity nu1|u| + nu3(c_s+c_A) + nu2 h max(0,-div u)
//                                                              (eq. RMnu)
//   max3    maximum over the 3x3x3 neighbourhood               (Section 6.1.1)
//   mean3   three-cell mean along x, y, z, floor, and its log  (Section 6.1.1)
//   edges   stresses, E, Lorentz edge products and heating on the three edge
//           sets (eqs. itv, nuij, ohm, vdiss, Joule)
//   cf      centre stresses / pressure and face energy fluxes (eqs. itv, ien,
//           ediffuse)
//   final   divergences -> F(f) (eqs. mass, mom, ien, indu), wall masking,
//           and the RK3 stage update dU <- alpha dU + F, f <- f + beta dt dU
//           (eqs. ddt, tupdate)
// Ghost planes of wall-bounded boxes are filled by the ghost kernels.
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

// Edge quantities.  At index (i, j, k):
//   z-edge (i-1/2, j-1/2, k): Gxy, Gyx, Ez, Lxz, Lyz, Qz
//   y-edge (i-1/2, j, k-1/2): Gxz, Gzx, Ey, Lxy, Lzy, Qy
//   x-edge (i, j-1/2, k-1/2): Gyz, Gzy, Ex, Lyx, Lzx, Qx
// G_ab = tau_ab - p_a u_b (momentum flux of component a along b, negated,
// plus the viscous stress); L the Lorentz edge products (used divided by mu);
// Q = 2 tau_ab S_ab + eta J^2 / mu (heating, interpolated to centres later).
template <class T>
__global__ __launch_bounds__(kBlock) void k_edges(const BoxDev* boxes, const Blk* tab, CP8<T> f,
                                                  const T* __restrict__ ux,
                                                  const T* __restrict__ uy,
                                                  const T* __restrict__ uz,
                                                  const T* __restrict__ lnt, Phys<T> ph,
                                                  P8<T> ez_, P8<T> ey_, P8<T> ex_) {
  CELL_PROLOGUE
  FIELD(R, f.p[0]);
  FIELD(PX, f.p[1]);
  FIELD(PY, f.p[2]);
  FIELD(PZ, f.p[3]);
  FIELD(BX, f.p[5]);
  FIELD(BY, f.p[6]);
  FIELD(BZ, f.p[7]);
  FIELD(UX, ux);
  FIELD(UY, uy);
  FIELD(UZ, uz);
  FIELD(LN, lnt);
  const unsigned tm = ph.terms;
  const bool visc = tm & T_VISC, res = tm & T_RESIST, ind = tm & T_INDUCT,
             lor = tm & T_LORENTZ, adv = tm & T_ADV;
  const bool need_nu = visc || (res && !(ph.eta_const > T(0)));
  const T inv_mu = ph.inv_mu;

  // ---- z-edge ----
  {
    T nxy = T(0), txy = T(0), sxy = T(0);
    if (need_nu) {
      auto lx = [&](int a, int b, int c) { return Xdn(g, LN, a, b, c); };
      nxy = fmax(g.dx, g.dy) * exp(Ydn(g, lx, i, j, k));
    }
    if (visc) {
      auto rx = [&](int a, int b, int c) { return Xdn(g, R, a, b, c); };
      const T rxy = Ydn(g, rx, i, j, k);
      sxy = T(0.5) * (DYdn(g, UX, i, j, k) + DXdn(g, UY, i, j, k));
      txy = rxy * nxy * sxy;
    }
    const T jz = DXdn(g, BY, i, j, k) - DYdn(g, BX, i, j, k);
    const T eta = ph.eta_const > T(0) ? ph.eta_const : ph.nuB * nxy;
    T ez = T(0);
    if (ind) ez = ez - (Ydn(g, UX, i, j, k) * Xdn(g, BY, i, j, k) - Xdn(g, UY, i, j, k) * Ydn(g, BX, i, j, k));
    if (res) ez = ez + eta * jz;
    T gxy = txy, gyx = txy;
    if (adv) {
      gxy = gxy - Ydn(g, PX, i, j, k) * Xdn(g, UY, i, j, k);
      gyx = gyx - Xdn(g, PY, i, j, k) * Ydn(g, UX, i, j, k);
    }
    T q = visc ? T(2) * txy * sxy : T(0);
    if (res) q = q + eta * jz * jz * inv_mu;
    ez_.p[0][o] = gxy;
    ez_.p[1][o] = gyx;
    ez_.p[2][o] = ez;
    ez_.p[3][o] = lor ? jz * Xdn(g, BY, i, j, k) : T(0);
    ez_.p[4][o] = lor ? jz * Ydn(g, BX, i, j, k) : T(0);
    ez_.p[5][o] = q;
  }
  // ---- y-edge ----
  {
    T nxz = T(0), txz = T(0), sxz = T(0);
    if (need_nu) {
      auto lx = [&](int a, int b, int c) { return Xdn(g, LN, a, b, c); };
      nxz = fmax(g.dx, g.dz) * exp(Zdn(g, lx, i, j, k));
    }
    if (visc) {
      auto rx = [&](int a, int b, int c) { return Xdn(g, R, a, b, c); };
      const T rxz = Zdn(g, rx, i, j, k);
      sxz = T(0.5) * (DZdn(g, UX, i, j, k) + DXdn(g, UZ, i, j, k));
      txz = rxz * nxz * sxz;
    }
    const T jy = DZdn(g, BX, i, j, k) - DXdn(g, BZ, i, j, k);
    const T eta = ph.eta_const > T(0) ? ph.eta_const : ph.nuB * nxz;
    T ey = T(0);
    if (ind) ey = ey - (Xdn(g, UZ, i, j, k) * Zdn(g, BX, i, j, k) - Zdn(g, UX, i, j, k) * Xdn(g, BZ, i, j, k));
    if (res) ey = ey + eta * jy;
    T gxz = txz, gzx = txz;
    if (adv) {
      gxz = gxz - Zdn(g, PX, i, j, k) * Xdn(g, UZ, i, j, k);
      gzx = gzx - Xdn(g, PZ, i, j, k) * Zdn(g, UX, i, j, k);
    }
    T q = visc ? T(2) * txz * sxz : T(0);
    if (res) q = q + eta * jy * jy * inv_mu;
    ey_.p[0][o] = gxz;
    ey_.p[1][o] = gzx;
    ey_.p[2][o] = ey;
    ey_.p[3][o] = lor ? jy * Xdn(g, BZ, i, j, k) : T(0);
    ey_.p[4][o] = lor ? jy * Zdn(g, BX, i, j, k) : T(0);
    ey_.p[5][o] = q;
  }
  // ---- x-edge ----
  {
    T nyz = T(0), tyz = T(0), syz = T(0);
    if (need_nu) {
      auto ly = [&](int a, int b, int c) { return Ydn(g, LN, a, b, c); };
      nyz = fmax(g.dy, g.dz) * exp(Zdn(g, ly, i, j, k));
    }
    if (visc) {
      auto ry = [&](int a, int b, int c) { return Ydn(g, R, a, b, c); };
      const T ryz = Zdn(g, ry, i, j, k);
      syz = T(0.5) * (DZdn(g, UY, i, j, k) + DYdn(g, UZ, i, j, k));
      tyz = ryz * nyz * syz;
    }
    const T jx = DYdn(g, BZ, i, j, k) - DZdn(g, BY, i, j, k);
    const T eta = ph.eta_const > T(0) ? ph.eta_const : ph.nuB * nyz;
    T ex = T(0);
    if (ind) ex = ex - (Zdn(g, UY, i, j, k) * Ydn(g, BZ, i, j, k) - Ydn(g, UZ, i, j, k) * Zdn(g, BY, i, j, k));
    if (res) ex = ex + eta * jx;
    T gyz = tyz, gzy = tyz;
    if (adv) {
      gyz = gyz - Zdn(g, PY, i, j, k) * Ydn(g, UZ, i, j, k);
      gzy = gzy - Ydn(g, PZ, i, j, k) * Zdn(g, UY, i, j, k);
    }
    T q = visc ? T(2) * tyz * syz : T(0);
    if (res) q = q + eta * jx * jx * inv_mu;
    ex_.p[0][o] = gyz;
    ex_.p[1][o] = gzy;
    ex_.p[2][o] = ex;
    ex_.p[3][o] = lor ? jx * Ydn(g, BZ, i, j, k) : T(0);
    ex_.p[4][o] = lor ? jx * Zdn(g, BY, i, j, k) : T(0);
    ex_.p[5][o] = q;
  }
}

// Centre and face quantities:
//   Gaa = tau_aa - aup(p_a) aup(u_a) - P   (centres; differentiated with ddadn)
//   Qc  = -P div u + sum_a tau_aa S_aa     (centres)
//   Ha  = -adn(e) u_a + nuE adn(rho) (dx_a adn(nu)) adn(e_m) ddadn(ln e_m)
//                                           (a-faces; differentiated with ddaup)
template <class T>
__global__ __launch_bounds__(kBlock) void k_cf(const BoxDev* boxes, const Blk* tab, CP8<T> f,
                                               const T* __restrict__ ux,
                                               const T* __restrict__ uy,
                                               const T* __restrict__ uz,
                                               const T* __restrict__ nt, Phys<T> ph, P8<T> out) {
  CELL_PROLOGUE
  FIELD(R, f.p[0]);
  FIELD(PX, f.p[1]);
  FIELD(PY, f.p[2]);
  FIELD(PZ, f.p[3]);
  FIELD(E, f.p[4]);
  FIELD(UX, ux);
  FIELD(UY, uy);
  FIELD(UZ, uz);
  FIELD(NT, nt);
  const unsigned tm = ph.terms;
  const T sxx = DXup(g, UX, i, j, k), syy = DYup(g, UY, i, j, k), szz = DZup(g, UZ, i, j, k);
  const T D = sxx + syy + szz;
  const T P = ph.gamma1 * f.p[4][o];
  const T r = f.p[0][o];
  T gxx = T(0), gyy = T(0), gzz = T(0), qc = T(0);
  if (tm & T_VISC) {
    const T n0 = nt[o];
    const T txx = r * (g.dx * n0) * (sxx + ph.c1 * D);
    const T tyy = r * (g.dy * n0) * (syy + ph.c1 * D);
    const T tzz = r * (g.dz * n0) * (szz + ph.c1 * D);
    gxx = txx;
    gyy = tyy;
    gzz = tzz;
    qc = txx * sxx + tyy * syy + tzz * szz;
  }
  if (tm & T_ADV) {
    gxx = gxx - Xup(g, PX, i, j, k) * Xup(g, UX, i, j, k);
    gyy = gyy - Yup(g, PY, i, j, k) * Yup(g, UY, i, j, k);
    gzz = gzz - Zup(g, PZ, i, j, k) * Zup(g, UZ, i, j, k);
  }
  if (tm & T_PRES) {
    gxx = gxx - P;
    gyy = gyy - P;
    gzz = gzz - P;
    qc = qc - P * D;
  }
  T hx = T(0), hy = T(0), hz = T(0);
  if (tm & T_ADV) {
    hx = -Xdn(g, E, i, j, k) * ux[o];
    hy = -Ydn(g, E, i, j, k) * uy[o];
    hz = -Zdn(g, E, i, j, k) * uz[o];
  }
  if (tm & T_EDIFF) {
    auto EM = [&](int a, int b, int c) -> T {
      const long long q = g.at(a, b, c);
      return f.p[4][q] / f.p[0][q];
    };
    auto LEM = [&](int a, int b, int c) -> T { return log(EM(a, b, c)); };
    hx = hx + ph.nuE * Xdn(g, R, i, j, k) * (g.dx * Xdn(g, NT, i, j, k)) * Xdn(g, EM, i, j, k) * DXdn(g, LEM, i, j, k);
    hy = hy + ph.nuE * Ydn(g, R, i, j, k) * (g.dy * Ydn(g, NT, i, j, k)) * Ydn(g, EM, i, j, k) * DYdn(g, LEM, i, j, k);
    hz = hz + ph.nuE * Zdn(g, R, i, j, k) * (g.dz * Zdn(g, NT, i, j, k)) * Zdn(g, EM, i, j, k) * DZdn(g, LEM, i, j, k);
  }
  out.p[0][o] = gxx;
  out.p[1][o] = gyy;
  out.p[2][o] = gzz;
  out.p[3][o] = qc;
  out.p[4][o] = hx;
  out.p[5][o] = hy;
  out.p[6][o] = hz;
}

// F(f) from the edge / centre / face quantities, wall masking, and either
// dfdt = F (f_out == nullptr) or the RK3 stage:
//   U = alpha dU_in + F   (U = F when dU_in == nullptr),
//   dU_out = U (if given),  f_out = f_in + bdt U.
template <class T>
__global__ __launch_bounds__(kBlock) void k_final(const BoxDev* boxes, const Blk* tab, CP8<T> f,
                                                  P8<T> ez_, P8<T> ey_, P8<T> ex_, P8<T> cf,
                                                  Phys<T> ph, CP8<T> du_in, P8<T> du_out,
                                                  P8<T> f_out, T alpha, T bdt) {
  CELL_PROLOGUE
  FIELD(R, f.p[0]);
  FIELD(PX, f.p[1]);
  FIELD(PY, f.p[2]);
  FIELD(PZ, f.p[3]);
  FIELD(GXY, ez_.p[0]);
  FIELD(GYX, ez_.p[1]);
  FIELD(EZ, ez_.p[2]);
  FIELD(LXZ, ez_.p[3]);
  FIELD(LYZ, ez_.p[4]);
  FIELD(QZ, ez_.p[5]);
  FIELD(GXZ, ey_.p[0]);
  FIELD(GZX, ey_.p[1]);
  FIELD(EY, ey_.p[2]);
  FIELD(LXY, ey_.p[3]);
  FIELD(LZY, ey_.p[4]);
  FIELD(QY, ey_.p[5]);
  FIELD(GYZ, ex_.p[0]);
  FIELD(GZY, ex_.p[1]);
  FIELD(EX, ex_.p[2]);
  FIELD(LYX, ex_.p[3]);
  FIELD(LZX, ex_.p[4]);
  FIELD(QX, ex_.p[5]);
  FIELD(GXX, cf.p[0]);
  FIELD(GYY, cf.p[1]);
  FIELD(GZZ, cf.p[2]);
  FIELD(HX, cf.p[4]);
  FIELD(HY, cf.p[5]);
  FIELD(HZ, cf.p[6]);
  const unsigned tm = ph.terms;
  const T inv_mu = ph.inv_mu;
  T F[8];
  F[0] = (tm & T_CONT) ? -(DXup(g, PX, i, j, k) + DYup(g, PY, i, j, k) + DZup(g, PZ, i, j, k)) : T(0);
  F[1] = DXdn(g, GXX, i, j, k) + DYup(g, GXY, i, j, k) + DZup(g, GXZ, i, j, k) +
         (Zup(g, LXY, i, j, k) - Yup(g, LXZ, i, j, k)) * inv_mu;
  F[2] = DYdn(g, GYY, i, j, k) + DZup(g, GYZ, i, j, k) + DXup(g, GYX, i, j, k) +
         (Xup(g, LYZ, i, j, k) - Zup(g, LYX, i, j, k)) * inv_mu;
  F[3] = DZdn(g, GZZ, i, j, k) + DXup(g, GZX, i, j, k) + DYup(g, GZY, i, j, k) +
         (Yup(g, LZX, i, j, k) - Xup(g, LZY, i, j, k)) * inv_mu;
  if (tm & T_GRAV) F[3] = F[3] - Zdn(g, R, i, j, k) * ph.gz;
  auto xqz = [&](int a, int b, int c) { return Xup(g, QZ, a, b, c); };
  auto xqy = [&](int a, int b, int c) { return Xup(g, QY, a, b, c); };
  auto yqx = [&](int a, int b, int c) { return Yup(g, QX, a, b, c); };
  F[4] = cf.p[3][o] + DXup(g, HX, i, j, k) + DYup(g, HY, i, j, k) + DZup(g, HZ, i, j, k) +
         Yup(g, xqz, i, j, k) + Zup(g, xqy, i, j, k) + Zup(g, yqx, i, j, k);
  F[5] = -(DYup(g, EZ, i, j, k) - DZup(g, EY, i, j, k));
  F[6] = -(DZup(g, EX, i, j, k) - DXup(g, EZ, i, j, k));
  F[7] = -(DXup(g, EY, i, j, k) - DYup(g, EX, i, j, k));
  if (g.wall) {
    const bool cen = k >= g.g0 && k < g.g1;
    const bool zf = k >= g.g0 && k <= g.g1;
    const bool pzok = k > g.g0 && k < g.g1;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const bool keep = v == 3 ? pzok : (v == 7 ? zf : cen);
      if (!keep) F[v] = T(0);
    }
  }
  if (f_out.p[0] == nullptr) {
#pragma unroll
    for (int v = 0; v < 8; ++v) du_out.p[v][o] = F[v];
    return;
  }
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const T U = du_in.p[0] ? alpha * du_in.p[v][o] + F[v] : F[v];
    if (du_out.p[0]) du_out.p[v][o] = U;
    f_out.p[v][o] = f.p[v][o] + bdt * U;
  }
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
template <class T>
void launch_stage(const Launch& L, const StageArgs<T>& a) {
  const dim3 grid(L.nblk), block(kBlock);
  L.at(PASS_PRIM);
  hipLaunchKernelGGL(k_prim<T>, grid, block, 0, L.stream, L.boxes, L.tab, a.f, a.w.ux, a.w.uy,
                     a.w.uz);
  L.at(PASS_NUS);
  hipLaunchKernelGGL(k_nus<T>, grid, block, 0, L.stream, L.boxes, L.tab, a.f, a.w.ux, a.w.uy,
                     a.w.uz, a.ph, a.w.nus);
  L.at(PASS_MAX3);
  hipLaunchKernelGGL(k_max3<T>, grid, block, 0, L.stream, L.boxes, L.tab, a.w.nus, a.w.nmax);
  L.at(PASS_MEAN3);
  hipLaunchKernelGGL(k_mean3<T>, grid, block, 0, L.stream, L.boxes, L.tab, a.w.nmax, a.w.nt,
                     a.w.lnt);
  L.at(PASS_EDGES);
  hipLaunchKernelGGL(k_edges<T>, grid, block, 0, L.stream, L.boxes, L.tab, a.f, a.w.ux, a.w.uy,
                     a.w.uz, a.w.lnt, a.ph, a.w.ez, a.w.ey, a.w.ex);
  L.at(PASS_CF);
  hipLaunchKernelGGL(k_cf<T>, grid, block, 0, L.stream, L.boxes, L.tab, a.f, a.w.ux, a.w.uy,
                     a.w.uz, a.w.nt, a.ph, a.w.cf);
  L.at(PASS_FINAL);
  hipLaunchKernelGGL(k_final<T>, grid, block, 0, L.stream, L.boxes, L.tab, a.f, a.w.ez, a.w.ey,
                     a.w.ex, a.w.cf, a.ph, a.du_in, a.du_out, a.f_out, a.alpha, a.bdt);
  L.at(PASS_END);
}

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

template void launch_stage<float>(const Launch&, const StageArgs<float>&);
template void launch_stage<double>(const Launch&, const StageArgs<double>&);
template void launch_nu<float>(const Launch&, CP8<float>, const Work<float>&, const Phys<float>&);
template void launch_nu<double>(const Launch&, CP8<double>, const Work<double>&, const Phys<double>&);
template void launch_ghost<float>(const Launch&, P8<float>);
template void launch_ghost<double>(const Launch&, P8<double>);

}  // namespace smhd
