// Device-side pieces shared by the stage kernels of mhd_zmarch.hip and
// mhd_zfinal.hip: the work-item loop, and the in-plane quantities of pass P
// (z-edge, centre and x/y-face terms), written once as point functions over
// an accessor of derived planes so that pass P (at its own columns) and
// pass F (on the halo strips of its divergences) evaluate the same
// expressions and round the same way.
#pragma once

#include "mhd_zmarch_api.hpp"

namespace smhd {

// Item loop of the stage kernels.  Grid mode (PERS false): one item
// per workgroup, blockIdx mapped XCD-aware.  Persistent mode: a grid of about
// one resident wave of workgroups; each pulls items from its XCD's queue
// (queue[x] counts the items of range x taken) and, once that is empty,
// from the other XCDs' ranges.  Results do not depend on the mode.
#define ZLOOP_BEGIN                                                            \
  __shared__ int snext_;                                                       \
  for (int item_ = zfirst<PERS>(nitems, queue, &snext_); item_ < nitems;      \
       item_ = znext<PERS>(nitems, queue, &snext_)) {                         \
  const ZItem it = items[item_];                                               \
  const BoxDev b = boxes[it.box];                                              \
  const Geo<T> g(b);                                                           \
  const int tx = (int)threadIdx.x % TX, ty = (int)threadIdx.x / TX;           \
  const int gx = wrapm(it.x0 + tx, b.nx), gy = wrapm(it.y0 + ty, b.ny);      \
  const bool own = (it.x0 + tx < b.nx) && (it.y0 + ty < b.ny);                \
  const int N = b.nzt;                                                         \
  const bool wall = b.wall != 0;                                               \
  const long long colo = b.off + (long long)gy * b.nx + gx;                   \
  const long long pstride = (long long)b.nx * b.ny;                           \
  auto valid = [&](int r_) { return !wall || (r_ >= 0 && r_ < N); };          \
  auto kk = [&](int r_) { return wall ? r_ : wrapm(r_, N); };                 \
  auto col = [&](int r_) { return colo + (long long)kk(r_) * pstride; };      \
  auto interior = [&](int r_) { return !wall || (r_ >= b.g0 && r_ < b.g1); };       \
  const T* __restrict__ zt = wall ? ztab + b.zoff : nullptr;                         \
  (void)zt;                                                                          \
  const T* __restrict__ zj_ = ztab + b.joff;                                         \
  auto zj = [&](int r_, int e_) { return zj_[(long long)kk(r_) * ZJ_COUNT + e_]; };  \
  (void)zj;

#define ZLOOP_END }

// Block maximum of a double (all threads call; result valid in thread 0).
template <int NT>
__device__ __forceinline__ double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  return sh[0];
}

// ---------------------------------------------------------------------------
// Field groups of pass F: bit v of a mask = field v is completed by that
// launch.  The stage runs one launch per mask of a set; each set partitions
// the 8 fields.  Split set: the momenta; rho and e; the magnetic field.
constexpr unsigned kFMasks[] = {0x0Eu, 0x11u, 0xE0u};
constexpr int kNFMasks = sizeof(kFMasks) / sizeof(kFMasks[0]);
template <unsigned FM> __host__ __device__ constexpr bool hasf(int v) { return (FM >> v) & 1u; }

// ---------------------------------------------------------------------------
// Derived in-plane inputs of pass P's quantities, by id: an accessor
// S(q, x, y) returns quantity q of the current z plane at tile position
// (x, y).  x-face quantities sit at (x - 1/2, y), y-face ones at (x, y - 1/2).
enum DQ : int {
  DQ_PX = 0, DQ_PY, DQ_E, DQ_BX, DQ_BY, DQ_LNT,   // the state and ln <nu>
  DQ_UX, DQ_UY,        // face velocities p_a / adn(rho)
  DQ_NU,               // <nu> = exp(ln <nu>)
  DQ_EM, DQ_LEM,       // e / rho and its log
  DQ_RXD, DQ_RYD,      // xdn(rho), ydn(rho)
  DQ_XL,               // xdn(ln <nu>)
  DQ_RHO,              // rho
  DQ_D,                // div u (from pass A1)
  DQ_LQ,               // ln(P / P_aver) (eq. pressure)
  DQ_COUNT
};

// z-directed edge (x - 1/2, y - 1/2): the edge viscosity (eq. nuij), the
// density ydn(xdn(rho)) and the strain S_xy (eq. itv).
template <class T, class A>
__device__ __forceinline__ T zedge_nu(const A& S, int x, int y, const Geo<T>& g) {
  return g.lxy * exp(op6<0, 0, T>([&](int m) { return S(DQ_XL, x, y + m); }, T(0)));
}
template <class T, class A> __device__ __forceinline__ T zedge_rho(const A& S, int x, int y) {
  return op6<0, 0, T>([&](int m) { return S(DQ_RXD, x, y + m); }, T(0));
}
// o2: from the second-order derivatives (the switch after eq. itv)
template <class T, class A>
__device__ __forceinline__ T zedge_strain(const A& S, int x, int y, const Geo<T>& g, bool o2 = false) {
  if (o2)
    return T(0.5) * ((S(DQ_UX, x, y) - S(DQ_UX, x, y - 1)) * g.hyi +
                     (S(DQ_UY, x, y) - S(DQ_UY, x - 1, y)) * g.hxi);
  return T(0.5) * (op6<1, 0, T>([&](int m) { return S(DQ_UX, x, y + m); }, g.hyi) +
                   op6<1, 0, T>([&](int m) { return S(DQ_UY, x + m, y); }, g.hxi));
}
// the viscous stress tau_xy = rho nu_xy S_xy on the z-edge
template <class T, class A>
__device__ __forceinline__ T zedge_tau(const A& S, int x, int y, const Geo<T>& g, bool o2 = false) {
  return zedge_rho<T>(S, x, y) * zedge_nu<T>(S, x, y, g) * zedge_strain<T>(S, x, y, g, o2);
}

// Second-order switch (Section 3 after eq. itv): per-cell flags of the
// positions whose strain takes the second-order derivatives (bit 0 the
// centre, 1 the x-edge, 2 the y-edge, 3 the z-edge of the cell's index).
enum : unsigned { RG_C = 1u, RG_XE = 2u, RG_YE = 4u, RG_ZE = 8u };

// z-directed edge: strain and stress (eq. itv; tq: the quenched stress, or
// null; o2: second-order strain), E_z (eq. ohm), the momentum fluxes G_xy = tau_xy - ydn(p_x)
// xdn(u_y) and G_yx = tau_xy - xdn(p_y) ydn(u_x), the Lorentz products L_xz =
// J_z xdn(B_y), L_yz = J_z ydn(B_x), and the heating 2 tau_xy S_xy +
// eta J_z^2 / mu (eq. vdiss, Joule).
template <class T, class A>
__device__ __forceinline__ void zedge_q(const A& S, int x, int y, const Geo<T>& g, const Phys<T>& ph,
                                        T& gxy, T& gyx, T& ez, T& lxz, T& lyz, T& qz,
                                        const T* tq = nullptr, bool o2 = false) {
  const unsigned tm = ph.terms;
  const bool visc = tm & T_VISC, res = tm & T_RESIST, ind = tm & T_INDUCT, lor = tm & T_LORENTZ,
             adv = tm & T_ADV;
  const bool need_nu = visc || (res && !(ph.eta_const > T(0)));
  T nxy = T(0), txy = T(0), sxy = T(0);
  if (need_nu) nxy = zedge_nu<T>(S, x, y, g);
  if (visc) {
    sxy = zedge_strain<T>(S, x, y, g, o2);
    txy = tq ? *tq : zedge_rho<T>(S, x, y) * nxy * sxy;
  }
  const T jz = op6<1, 0, T>([&](int m) { return S(DQ_BY, x + m, y); }, g.hxi) -
               op6<1, 0, T>([&](int m) { return S(DQ_BX, x, y + m); }, g.hyi);
  const T eta = ph.eta_const > T(0) ? ph.eta_const : ph.nuB * nxy;
  const T xBY = op6<0, 0, T>([&](int m) { return S(DQ_BY, x + m, y); }, T(0));
  const T yBX = op6<0, 0, T>([&](int m) { return S(DQ_BX, x, y + m); }, T(0));
  const T yUX = op6<0, 0, T>([&](int m) { return S(DQ_UX, x, y + m); }, T(0));
  const T xUY = op6<0, 0, T>([&](int m) { return S(DQ_UY, x + m, y); }, T(0));
  T e_ = T(0);
  if (ind) e_ = e_ - (yUX * xBY - xUY * yBX);
  if (res) e_ = e_ + eta * jz;
  T a = txy, c = txy;
  if (adv) {
    a = a - op6<0, 0, T>([&](int m) { return S(DQ_PX, x, y + m); }, T(0)) * xUY;
    c = c - op6<0, 0, T>([&](int m) { return S(DQ_PY, x + m, y); }, T(0)) * yUX;
  }
  T q = visc ? T(2) * txy * sxy : T(0);
  if (res) q = q + eta * jz * jz * ph.inv_mu;
  gxy = a;
  gyx = c;
  ez = e_;
  lxz = lor ? jz * xBY : T(0);
  lyz = lor ? jz * yBX : T(0);
  qz = q;
}

// Cell centre (x, y): the strain S_xx, S_yy and the viscous stress tau_xx =
// rho nu_xx (S_xx + c1 div u), tau_yy (eq. itv, eq. nuij); with o2 from the
// second-order derivatives and D2, the second-order div u.
template <class T, class A>
__device__ __forceinline__ void centre_tau(const A& S, int x, int y, const Geo<T>& g, const Phys<T>& ph,
                                           T& sxx, T& syy, T& txx, T& tyy, bool o2 = false,
                                           T D2 = T(0)) {
  if (o2) {
    sxx = (S(DQ_UX, x + 1, y) - S(DQ_UX, x, y)) * g.hxi;
    syy = (S(DQ_UY, x, y + 1) - S(DQ_UY, x, y)) * g.hyi;
  } else {
    sxx = op6<1, 1, T>([&](int m) { return S(DQ_UX, x + m, y); }, g.hxi);
    syy = op6<1, 1, T>([&](int m) { return S(DQ_UY, x, y + m); }, g.hyi);
  }
  const T Dc = o2 ? D2 : S(DQ_D, x, y);
  const T rn = S(DQ_RHO, x, y) * S(DQ_NU, x, y);
  txx = rn * g.lx * (sxx + ph.c1 * Dc);
  tyy = rn * g.ly * (syy + ph.c1 * Dc);
}

// Cell centre: G_xx = tau_xx - xup(p_x) xup(u_x), G_yy likewise (eq. itv,
// eq. mom), and Q_c = tau_xx S_xx + tau_yy S_yy - P div u (eq. vdiss, eq.
// ien); tq: the quenched tau_xx and tau_yy (tq[0], tq[stride]), or null.
template <class T, class A>
__device__ __forceinline__ void centre_q(const A& S, int x, int y, const Geo<T>& g, const Phys<T>& ph,
                                         T& gxx, T& gyy, T& qc, const T* tq = nullptr,
                                         long long stride = 0, bool o2 = false, T D2 = T(0)) {
  const unsigned tm = ph.terms;
  const bool visc = tm & T_VISC, adv = tm & T_ADV, pres = tm & T_PRES;
  T sxx, syy, txx, tyy;
  centre_tau<T>(S, x, y, g, ph, sxx, syy, txx, tyy, o2, D2);
  const T Dc = S(DQ_D, x, y);
  const T Pc = ph.gamma1 * S(DQ_E, x, y);
  T a = T(0), c = T(0), q = T(0);
  if (visc) {
    if (tq) {
      txx = tq[0];
      tyy = tq[stride];
    }
    a = txx;
    c = tyy;
    q = txx * sxx + tyy * syy;
  }
  if (adv) {
    a = a - op6<0, 1, T>([&](int m) { return S(DQ_PX, x + m, y); }, T(0)) *
                op6<0, 1, T>([&](int m) { return S(DQ_UX, x + m, y); }, T(0));
    c = c - op6<0, 1, T>([&](int m) { return S(DQ_PY, x, y + m); }, T(0)) *
                op6<0, 1, T>([&](int m) { return S(DQ_UY, x, y + m); }, T(0));
  }
  if (pres) q = q - Pc * Dc;
  gxx = a;
  gyy = c;
  qc = q;
}

// x-face (x - 1/2, y): the energy flux H_x = -xdn(e) u_x + nuE xdn(rho)
// (l_x xdn(nu)) xdn(e_m) ddxdn(ln e_m) (eq. ien, eq. ediffuse).
template <class T, class A>
__device__ __forceinline__ T xface_h(const A& S, int x, int y, const Geo<T>& g, const Phys<T>& ph) {
  const unsigned tm = ph.terms;
  T h = T(0);
  if (tm & T_ADV) h = -op6<0, 0, T>([&](int m) { return S(DQ_E, x + m, y); }, T(0)) * S(DQ_UX, x, y);
  if (tm & T_EDIFF)
    h = h + ph.nuE * S(DQ_RXD, x, y) *
                (g.lx * op6<0, 0, T>([&](int m) { return S(DQ_NU, x + m, y); }, T(0))) *
                op6<0, 0, T>([&](int m) { return S(DQ_EM, x + m, y); }, T(0)) *
                op6<1, 0, T>([&](int m) { return S(DQ_LEM, x + m, y); }, g.hxi);
  return h;
}

template <class T, class A>
__device__ __forceinline__ T yface_h(const A& S, int x, int y, const Geo<T>& g, const Phys<T>& ph) {
  const unsigned tm = ph.terms;
  T h = T(0);
  if (tm & T_ADV) h = -op6<0, 0, T>([&](int m) { return S(DQ_E, x, y + m); }, T(0)) * S(DQ_UY, x, y);
  if (tm & T_EDIFF)
    h = h + ph.nuE * S(DQ_RYD, x, y) *
                (g.ly * op6<0, 0, T>([&](int m) { return S(DQ_NU, x, y + m); }, T(0))) *
                op6<0, 0, T>([&](int m) { return S(DQ_EM, x, y + m); }, T(0)) *
                op6<1, 0, T>([&](int m) { return S(DQ_LEM, x, y + m); }, g.hyi);
  return h;
}

// Pressure gradients on the x- and y-faces, kept out of the fluxes (with
// the sign of a gradient that pass F subtracts): gamma1 ddadn(e), or with
// T_LNP the form of eq. pressure, exp(ln P_aver) exp(adn(q)) ddadn(q) with
// q = ln(P / P_aver) (the plane mean has no x or y derivative; epa =
// exp(ln P_aver) of the plane).  With T_CORI the in-plane parts of the
// Coriolis force -2 Omega x p (eq. mom) are added: +2 Omega_z p_y on
// x-faces, -2 Omega_z p_x on y-faces.
template <class T, class A>
__device__ __forceinline__ void face_dp(const A& S, int x, int y, const Geo<T>& g, const Phys<T>& ph, T epa,
                                        T& dpx, T& dpy) {
  const unsigned tm = ph.terms;
  T a = T(0), c = T(0);
  if ((tm & T_PRES) && (tm & T_LNP)) {
    a = epa * exp(op6<0, 0, T>([&](int m) { return S(DQ_LQ, x + m, y); }, T(0))) *
        op6<1, 0, T>([&](int m) { return S(DQ_LQ, x + m, y); }, g.hxi);
    c = epa * exp(op6<0, 0, T>([&](int m) { return S(DQ_LQ, x, y + m); }, T(0))) *
        op6<1, 0, T>([&](int m) { return S(DQ_LQ, x, y + m); }, g.hyi);
  } else if (tm & T_PRES) {
    a = ph.gamma1 * op6<1, 0, T>([&](int m) { return S(DQ_E, x + m, y); }, g.hxi);
    c = ph.gamma1 * op6<1, 0, T>([&](int m) { return S(DQ_E, x, y + m); }, g.hyi);
  }
  if (tm & T_CORI) {
    a -= ph.cor2[2] * op6<0, 0, T>([&](int m) {
           return op6<0, 1, T>([&](int n) { return S(DQ_PY, x + m, y + n); }, T(0));
         }, T(0));
    c += ph.cor2[2] * op6<0, 0, T>([&](int n) {
           return op6<0, 1, T>([&](int m) { return S(DQ_PX, x + m, y + n); }, T(0));
         }, T(0));
  }
  dpx = a;
  dpy = c;
}

}  // namespace smhd
