// Discrete adjoint of the right-hand side (see mhd_adjoint.hpp): the program
// builder (host) and the forward / transposed whole-box kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "mhd_adjoint.hpp"

namespace smhd {

// ---------------------------------------------------------------------------
// Program builder.  Follows the right-hand side of eqs. mass, mom, ien, indu,
// ohm, itv, vdiss, RMnu, nuij and ediffuse term by term, with the readings
// of the float64 reference (dissipative viscous sign, eta a magnetic
// diffusivity, shock viscosity nu2 h max(0, -div u), edge viscosities by
// averaging ln nu, the energy-diffusion flux without the extra grid step).
namespace {

constexpr int ZERO = -1;   // the zero field: never stored, folded away

struct Builder {
  VProgram P;

  int emit(int op, int a, int b, int c, double k, int geo, int ax, int fam, int form) {
    VInstr I{};
    I.op = op;
    I.out = P.nslots++;
    I.a = a;
    I.b = b;
    I.c = c;
    I.k = k;
    I.geo = geo;
    I.ax = ax;
    I.fam = fam;
    I.form = form;
    P.code.push_back(I);
    return I.out;
  }
  int un(int op, int a, double k = 0.0, int geo = G_ONE) {
    return emit(op, a, ZERO, ZERO, k, geo, 0, 0, 0);
  }
  int st(int a, int ax, int fam, int form) {
    return a == ZERO ? ZERO : emit(V_STEN, a, ZERO, ZERO, 0.0, G_ONE, ax, fam, form);
  }
  // staggered operators (eqs. deriv, interp): fam 0 interpolation, 1 derivative
  int xdn(int a) { return st(a, VX, 0, 0); }
  int xup(int a) { return st(a, VX, 0, 1); }
  int ydn(int a) { return st(a, VY, 0, 0); }
  int yup(int a) { return st(a, VY, 0, 1); }
  int zdn(int a) { return st(a, VZ, 0, 0); }
  int zup(int a) { return st(a, VZ, 0, 1); }
  int ddxdn(int a) { return st(a, VX, 1, 0); }
  int ddxup(int a) { return st(a, VX, 1, 1); }
  int ddydn(int a) { return st(a, VY, 1, 0); }
  int ddyup(int a) { return st(a, VY, 1, 1); }
  int ddzdn(int a) { return st(a, VZ, 1, 0); }
  int ddzup(int a) { return st(a, VZ, 1, 1); }

  int neg(int a) { return a == ZERO ? ZERO : un(V_SCALE, a, -1.0); }
  int add(int a, int b) {
    if (a == ZERO) return b;
    if (b == ZERO) return a;
    return emit(V_ADD, a, b, ZERO, 0.0, G_ONE, 0, 0, 0);
  }
  int sub(int a, int b) {
    if (b == ZERO) return a;
    if (a == ZERO) return neg(b);
    return emit(V_SUB, a, b, ZERO, 0.0, G_ONE, 0, 0, 0);
  }
  int mul(int a, int b) {
    if (a == ZERO || b == ZERO) return ZERO;
    return emit(V_MUL, a, b, ZERO, 0.0, G_ONE, 0, 0, 0);
  }
  int div(int a, int b) {   // b is never the zero field
    if (a == ZERO) return ZERO;
    return emit(V_DIV, a, b, ZERO, 0.0, G_ONE, 0, 0, 0);
  }
  int scale(int a, double k, int geo = G_ONE) { return a == ZERO ? ZERO : un(V_SCALE, a, k, geo); }
  int divc(int a, double k) { return a == ZERO ? ZERO : un(V_DIVC, a, k); }
  int fsqrt(int a) { return un(V_SQRT, a); }
  int flog(int a) { return un(V_LOG, a); }
  int fexp(int a) { return un(V_EXP, a); }
  int relu(int a) { return a == ZERO ? ZERO : un(V_RELU, a); }
  int floor_at(int a, double k) { return un(V_FLOOR, a, k); }
  int norm3(int a, int b, int c) { return emit(V_NORM3, a, b, c, 0.0, G_ONE, 0, 0, 0); }
  int max3(int a, int ax) { return emit(V_MAX3, a, ZERO, ZERO, 0.0, G_ONE, ax, 0, 0); }
  int mean3(int a, int ax) { return emit(V_MEAN3, a, ZERO, ZERO, 0.0, G_ONE, ax, 0, 0); }
  int fill(double k, int geo = G_ONE) { return emit(V_FILL, ZERO, ZERO, ZERO, k, geo, 0, 0, 0); }
  int fabs_(int a) { return un(V_ABS, a); }
  int d2(int a, int ax) { return emit(V_D2, a, ZERO, ZERO, 0.0, G_ONE, ax, 0, 0); }
  int sdiv(int a, int b) { return emit(V_SDIV, a, b, ZERO, 0.0, G_ONE, 0, 0, 0); }
  int cap(int a, double k) { return un(V_CAP, a, k); }
  // second-order staggered derivative (form 0 dn, 1 up)
  int dd2(int a, int ax, int form) { return emit(V_STEN, a, ZERO, ZERO, 0.0, G_ONE, ax, 2, form); }
  // 1 where a cell touching position `kind` is rough, else 0 (no derivative)
  int rough(int lnr, int lne, double lim, int kind) {
    return emit(V_ROUGH, lnr, lne, ZERO, lim, G_ONE, kind, 0, 0);
  }
  int sel(int a, int b, int m) { return emit(V_SEL, a, b, m, 0.0, G_ONE, 0, 0, 0); }
  int pmean(int a) { return emit(V_PMEAN, a, ZERO, ZERO, 0.0, G_ONE, 0, 0, 0); }
};

// Drops instructions whose results never reach an output, renumbers slots
// densely (0..7 stay the state) and makes every output a slot of its own
// that no instruction reads.
VProgram finish(Builder& B, int out[8]) {
  for (int v = 0; v < 8; ++v) {
    if (out[v] == ZERO) out[v] = B.fill(0.0);
    bool shared = out[v] < 8;
    for (int w = 0; w < v; ++w) shared |= out[w] == out[v];
    for (const auto& I : B.P.code) shared |= I.a == out[v] || I.b == out[v] || I.c == out[v];
    if (shared) out[v] = B.un(V_SCALE, out[v], 1.0);
  }
  VProgram& P = B.P;
  std::vector<char> live(P.nslots, 0);
  for (int v = 0; v < 8; ++v) live[out[v]] = 1;
  std::vector<char> keep(P.code.size(), 0);
  for (int n = (int)P.code.size() - 1; n >= 0; --n) {
    const VInstr& I = P.code[n];
    if (!live[I.out]) continue;
    keep[n] = 1;
    for (int s : {I.a, I.b, I.c})
      if (s >= 0) live[s] = 1;
  }
  std::vector<int> remap(P.nslots, -1);
  for (int s = 0; s < 8; ++s) remap[s] = s;
  VProgram R;
  R.nslots = 8;
  for (size_t n = 0; n < P.code.size(); ++n) {
    if (!keep[n]) continue;
    VInstr I = P.code[n];
    remap[I.out] = R.nslots++;
    I.out = remap[I.out];
    I.a = I.a >= 0 ? remap[I.a] : ZERO;
    I.b = I.b >= 0 ? remap[I.b] : ZERO;
    I.c = I.c >= 0 ? remap[I.c] : ZERO;
    R.code.push_back(I);
  }
  for (int v = 0; v < 8; ++v) R.out[v] = remap[out[v]];
  return R;
}

}  // namespace

VProgram build_rhs_program(const mhd_params& p, double dt) {
  Builder B;
  const unsigned T = p.terms;
  const int rho = 0, px = 1, py = 2, pz = 3, e = 4, bx = 5, by = 6, bz = 7;
  const int Z = ZERO;

  // primitives and the smoothed viscosity (Section 6.1.1, eq. RMnu)
  const int P = B.scale(e, p.gamma - 1.0);
  const int ux = B.div(px, B.xdn(rho)), uy = B.div(py, B.ydn(rho)), uz = B.div(pz, B.zdn(rho));
  const int sxx = B.ddxup(ux), syy = B.ddyup(uy), szz = B.ddzup(uz);
  const int D = B.add(B.add(sxx, syy), szz);
  int nus;
  if (p.nu_const > 0) {
    nus = B.fill(p.nu_const, G_HINV);
  } else {
    const int ub = B.norm3(B.xup(ux), B.yup(uy), B.zup(uz));
    const int bb = B.norm3(B.xup(bx), B.yup(by), B.zup(bz));
    const int cs = B.fsqrt(B.div(B.scale(P, p.gamma), rho));
    const int ca = B.div(bb, B.fsqrt(B.scale(rho, p.mu)));
    nus = B.add(B.add(B.scale(ub, p.nu1), B.scale(B.add(cs, ca), p.nu3)),
                B.scale(B.relu(B.neg(D)), p.nu2, G_H));
    // Smagorinsky viscosity (eq. nusmag): the strain of eq. itv, its edge
    // components interpolated to the centre
    if (T & MHD_T_SMAG) {
      const int cxy = B.yup(B.xup(B.scale(B.add(B.ddydn(ux), B.ddxdn(uy)), 0.5)));
      const int cxz = B.zup(B.xup(B.scale(B.add(B.ddzdn(ux), B.ddxdn(uz)), 0.5)));
      const int cyz = B.zup(B.yup(B.scale(B.add(B.ddzdn(uy), B.ddydn(uz)), 0.5)));
      const int dia = B.add(B.add(B.mul(sxx, sxx), B.mul(syy, syy)), B.mul(szz, szz));
      const int off = B.add(B.add(B.mul(cxy, cxy), B.mul(cxz, cxz)), B.mul(cyz, cyz));
      const int s2 = B.scale(B.add(B.sub(dia, B.scale(B.mul(D, D), 1.0 / 3.0)), B.scale(off, 2.0)), 2.0);
      nus = B.add(nus, B.scale(B.fsqrt(B.relu(s2)), p.c_smag, G_H));
    }
  }
  // maximum over three (or, with MHD_T_MAX5, five) cells along each axis
  auto mx = [&](int a, int ax) { return T & MHD_T_MAX5 ? B.max3(B.max3(a, ax), ax) : B.max3(a, ax); };
  int m = mx(mx(mx(nus, VX), VY), VZ);
  int nt = B.mean3(B.mean3(B.mean3(m, VX), VY), VZ);
  nt = B.floor_at(nt, 1e-30);
  const int em = B.div(e, rho);
  const int lnt = B.flog(nt);

  // edge viscosities and densities (eq. nuij)
  const int nxy = B.scale(B.fexp(B.ydn(B.xdn(lnt))), 1.0, G_LXY);
  const int nxz = B.scale(B.fexp(B.zdn(B.xdn(lnt))), 1.0, G_LXZ);
  const int nyz = B.scale(B.fexp(B.zdn(B.ydn(lnt))), 1.0, G_LYZ);
  const int rxy = B.ydn(B.xdn(rho)), rxz = B.zdn(B.xdn(rho)), ryz = B.zdn(B.ydn(rho));

  // strain and stress (eq. itv)
  int vxx = sxx, vyy = syy, vzz = szz, Dt = D;
  int vxy = B.scale(B.add(B.ddydn(ux), B.ddxdn(uy)), 0.5);
  int vxz = B.scale(B.add(B.ddzdn(ux), B.ddxdn(uz)), 0.5);
  int vyz = B.scale(B.add(B.ddzdn(uy), B.ddydn(uz)), 0.5);
  // second-order switch (Section 3 after eq. itv): where a touching cell is
  // rough, the stress's strain and div u from second-order derivatives
  if ((T & MHD_T_ORDER2) && (T & MHD_T_VISC)) {
    const int lnr = B.flog(rho), lne = B.flog(em);
    const int mc = B.rough(lnr, lne, p.d2_lim, 0), mxe = B.rough(lnr, lne, p.d2_lim, 1);
    const int mye = B.rough(lnr, lne, p.d2_lim, 2), mze = B.rough(lnr, lne, p.d2_lim, 3);
    const int s2xx = B.dd2(ux, VX, 1), s2yy = B.dd2(uy, VY, 1), s2zz = B.dd2(uz, VZ, 1);
    Dt = B.sel(D, B.add(B.add(s2xx, s2yy), s2zz), mc);
    vxx = B.sel(vxx, s2xx, mc);
    vyy = B.sel(vyy, s2yy, mc);
    vzz = B.sel(vzz, s2zz, mc);
    vxy = B.sel(vxy, B.scale(B.add(B.dd2(ux, VY, 0), B.dd2(uy, VX, 0)), 0.5), mze);
    vxz = B.sel(vxz, B.scale(B.add(B.dd2(ux, VZ, 0), B.dd2(uz, VX, 0)), 0.5), mye);
    vyz = B.sel(vyz, B.scale(B.add(B.dd2(uy, VZ, 0), B.dd2(uz, VY, 0)), 0.5), mxe);
  }
  int txx = B.mul(B.mul(rho, B.scale(nt, 1.0, G_LX)), B.add(vxx, B.scale(Dt, p.c1)));
  int tyy = B.mul(B.mul(rho, B.scale(nt, 1.0, G_LY)), B.add(vyy, B.scale(Dt, p.c1)));
  int tzz = B.mul(B.mul(rho, B.scale(nt, 1.0, G_LZ)), B.add(vzz, B.scale(Dt, p.c1)));
  int txy = B.mul(B.mul(rxy, nxy), vxy);
  int txz = B.mul(B.mul(rxz, nxz), vxz);
  int tyz = B.mul(B.mul(ryz, nyz), vyz);
  // quenching (Section 6.2, eq. quench): each component times
  // min(max over 3x3x3 of D2 / (|tau| + D2 / q_max), q_lim)
  if ((T & MHD_T_QUENCH) && (T & MHD_T_VISC)) {
    auto quench = [&](int t) {
      const int s = B.add(B.add(B.fabs_(B.d2(t, VX)), B.fabs_(B.d2(t, VY))), B.fabs_(B.d2(t, VZ)));
      const int q = B.sdiv(s, B.add(B.fabs_(t), B.divc(s, p.q_max)));
      return B.mul(t, B.cap(B.max3(B.max3(B.max3(q, VX), VY), VZ), p.q_lim));
    };
    txx = quench(txx);
    tyy = quench(tyy);
    tzz = quench(tzz);
    txy = quench(txy);
    txz = quench(txz);
    tyz = quench(tyz);
  }

  // current and electric field (eq. ohm)
  const int jx = B.sub(B.ddydn(bz), B.ddzdn(by));
  const int jy = B.sub(B.ddzdn(bx), B.ddxdn(bz));
  const int jz = B.sub(B.ddxdn(by), B.ddydn(bx));
  int etx, ety, etz;
  if (p.eta_const > 0) {
    etx = ety = etz = B.fill(p.eta_const);
  } else {
    etx = B.scale(nyz, p.nuB);
    ety = B.scale(nxz, p.nuB);
    etz = B.scale(nxy, p.nuB);
  }
  int ex = Z, ey = Z, ez = Z;
  if (T & MHD_T_INDUCT) {
    ex = B.sub(ex, B.sub(B.mul(B.zdn(uy), B.ydn(bz)), B.mul(B.ydn(uz), B.zdn(by))));
    ey = B.sub(ey, B.sub(B.mul(B.xdn(uz), B.zdn(bx)), B.mul(B.zdn(ux), B.xdn(bz))));
    ez = B.sub(ez, B.sub(B.mul(B.ydn(ux), B.xdn(by)), B.mul(B.xdn(uy), B.ydn(bx))));
  }
  if (T & MHD_T_RESIST) {
    ex = B.add(ex, B.mul(etx, jx));
    ey = B.add(ey, B.mul(ety, jy));
    ez = B.add(ez, B.mul(etz, jz));
  }

  // mass (eq. mass)
  int drho = Z;
  if (T & MHD_T_CONT) drho = B.neg(B.add(B.add(B.ddxup(px), B.ddyup(py)), B.ddzup(pz)));

  // momentum (eq. mom)
  int dpx = Z, dpy = Z, dpz = Z;
  if (T & MHD_T_ADV) {
    dpx = B.sub(dpx, B.add(B.add(B.ddxdn(B.mul(B.xup(px), B.xup(ux))),
                                 B.ddyup(B.mul(B.ydn(px), B.xdn(uy)))),
                           B.ddzup(B.mul(B.zdn(px), B.xdn(uz)))));
    dpy = B.sub(dpy, B.add(B.add(B.ddydn(B.mul(B.yup(py), B.yup(uy))),
                                 B.ddzup(B.mul(B.zdn(py), B.ydn(uz)))),
                           B.ddxup(B.mul(B.xdn(py), B.ydn(ux)))));
    dpz = B.sub(dpz, B.add(B.add(B.ddzdn(B.mul(B.zup(pz), B.zup(uz))),
                                 B.ddxup(B.mul(B.xdn(pz), B.zdn(ux)))),
                           B.ddyup(B.mul(B.ydn(pz), B.zdn(uy)))));
  }
  if (T & MHD_T_PRES) {
    if (T & MHD_T_LNP) {
      // eq. pressure: exp(adn ln P_aver) exp(adn q) (ddadn q + ddadn ln P_aver),
      // q = ln(P / P_aver), P_aver the mean of P over each z plane
      const int lpa = B.flog(B.pmean(P));
      const int q = B.sub(B.flog(P), lpa);
      auto g = [&](int ax) {
        return B.mul(B.mul(B.fexp(B.st(lpa, ax, 0, 0)), B.fexp(B.st(q, ax, 0, 0))),
                     B.add(B.st(q, ax, 1, 0), B.st(lpa, ax, 1, 0)));
      };
      dpx = B.sub(dpx, g(VX));
      dpy = B.sub(dpy, g(VY));
      dpz = B.sub(dpz, g(VZ));
    } else {
      dpx = B.sub(dpx, B.ddxdn(P));
      dpy = B.sub(dpy, B.ddydn(P));
      dpz = B.sub(dpz, B.ddzdn(P));
    }
  }
  if (T & MHD_T_LORENTZ) {
    dpx = B.add(dpx, B.divc(B.sub(B.zup(B.mul(jy, B.xdn(bz))), B.yup(B.mul(jz, B.xdn(by)))), p.mu));
    dpy = B.add(dpy, B.divc(B.sub(B.xup(B.mul(jz, B.ydn(bx))), B.zup(B.mul(jx, B.ydn(bz)))), p.mu));
    dpz = B.add(dpz, B.divc(B.sub(B.yup(B.mul(jx, B.zdn(by))), B.xup(B.mul(jy, B.zdn(bx)))), p.mu));
  }
  if (T & MHD_T_VISC) {
    dpx = B.add(B.add(B.add(dpx, B.ddxdn(txx)), B.ddyup(txy)), B.ddzup(txz));
    dpy = B.add(B.add(B.add(dpy, B.ddydn(tyy)), B.ddzup(tyz)), B.ddxup(txy));
    dpz = B.add(B.add(B.add(dpz, B.ddzdn(tzz)), B.ddxup(txz)), B.ddyup(tyz));
  }
  if (T & MHD_T_GRAV) dpz = B.sub(dpz, B.scale(B.zdn(rho), p.gz));
  // Coriolis force (eq. mom): -2 Omega x p, each component on its own face
  if (T & MHD_T_CORI) {
    const double wx = 2.0 * p.omega[0], wy = 2.0 * p.omega[1], wz = 2.0 * p.omega[2];
    auto term = [&](int acc, int v, double w) { return w == 0.0 ? acc : B.add(acc, B.scale(v, w)); };
    dpx = term(term(dpx, B.xdn(B.zup(pz)), -wy), B.xdn(B.yup(py)), wz);
    dpy = term(term(dpy, B.ydn(B.xup(px)), -wz), B.ydn(B.zup(pz)), wx);
    dpz = term(term(dpz, B.zdn(B.yup(py)), -wx), B.zdn(B.xup(px)), wy);
  }

  // internal energy (eqs. ien, vdiss, ediffuse)
  int de = Z;
  if (T & MHD_T_ADV)
    de = B.sub(de, B.add(B.add(B.ddxup(B.mul(B.xdn(e), ux)), B.ddyup(B.mul(B.ydn(e), uy))),
                         B.ddzup(B.mul(B.zdn(e), uz))));
  if (T & MHD_T_PRES) de = B.sub(de, B.mul(P, D));
  if (T & MHD_T_VISC) {
    int qv = B.add(B.add(B.mul(txx, vxx), B.mul(tyy, vyy)), B.mul(tzz, vzz));
    qv = B.add(qv, B.scale(B.add(B.add(B.yup(B.xup(B.mul(txy, vxy))), B.zup(B.xup(B.mul(txz, vxz)))),
                                 B.zup(B.yup(B.mul(tyz, vyz)))),
                           2.0));
    de = B.add(de, qv);
  }
  if (T & MHD_T_RESIST) {
    const int qj = B.divc(B.add(B.add(B.zup(B.yup(B.mul(B.mul(etx, jx), jx))),
                                      B.zup(B.xup(B.mul(B.mul(ety, jy), jy)))),
                                B.yup(B.xup(B.mul(B.mul(etz, jz), jz)))),
                          p.mu);
    de = B.add(de, qj);
  }
  if (T & MHD_T_EDIFF) {
    const int lne = B.flog(em);
    const int fx = B.mul(B.mul(B.mul(B.scale(B.xdn(rho), p.nuE), B.scale(B.xdn(nt), 1.0, G_LX)), B.xdn(em)),
                         B.ddxdn(lne));
    const int fy = B.mul(B.mul(B.mul(B.scale(B.ydn(rho), p.nuE), B.scale(B.ydn(nt), 1.0, G_LY)), B.ydn(em)),
                         B.ddydn(lne));
    // eq. ediffav: the z flux differentiates ln e_m - ln <e_m>_horiz
    const int lnez = (T & MHD_T_EDIFFAV) ? B.sub(lne, B.flog(B.pmean(em))) : lne;
    const int fz = B.mul(B.mul(B.mul(B.scale(B.zdn(rho), p.nuE), B.scale(B.zdn(nt), 1.0, G_LZF)), B.zdn(em)),
                         B.ddzdn(lnez));
    de = B.add(B.add(B.add(de, B.ddxup(fx)), B.ddyup(fy)), B.ddzup(fz));
  }
  // Newtonian cooling (eq. NewtonCool, eq. rhocool)
  if (T & MHD_T_COOL) {
    int q = B.scale(B.mul(rho, B.sub(em, B.fill(p.e_cool))), -1.0 / p.t_cool);
    if (p.cool_cut == 1 || p.cool_cut == 2) {
      const int r = B.scale(rho, 1.0 / p.rho_cool);
      const int r2 = B.mul(r, r);
      const int den = B.add(B.fill(1.0), r2);
      q = B.mul(q, B.div(p.cool_cut == 1 ? r2 : B.fill(1.0), den));
    }
    de = B.add(de, q);
  }

  // induction (eq. indu)
  int dbx = B.neg(B.sub(B.ddyup(ez), B.ddzup(ey)));
  int dby = B.neg(B.sub(B.ddzup(ex), B.ddxup(ez)));
  int dbz = B.neg(B.sub(B.ddxup(ey), B.ddyup(ex)));
  // div B diffusion c_divb h_min^2 / dt grad(div B), with the step's dt
  if ((T & MHD_T_DIVB) && dt > 0.0) {
    const int divb = B.add(B.add(B.ddxup(bx), B.ddyup(by)), B.ddzup(bz));
    auto kd = [&](int a) { return B.scale(B.scale(a, p.c_divb / dt, G_HMIN), 1.0, G_HMIN); };
    dbx = B.add(dbx, kd(B.ddxdn(divb)));
    dby = B.add(dby, kd(B.ddydn(divb)));
    dbz = B.add(dbz, kd(B.ddzdn(divb)));
  }

  int out[8] = {drho, dpx, dpy, dpz, de, dbx, dby, dbz};
  return finish(B, out);
}

// ---------------------------------------------------------------------------
// Storage plan.
VPlan plan_program(const VProgram& P) {
  const int n = (int)P.code.size(), S = P.nslots;
  // values some transpose reads: stored, never recycled
  std::vector<char> keep(S, 0);
  for (int s = 0; s < 8; ++s) keep[s] = 1;
  for (const VInstr& I : P.code) {
    switch (I.op) {
      case V_MUL: keep[I.a] = keep[I.b] = 1; break;
      case V_DIV: keep[I.b] = keep[I.out] = 1; break;
      case V_SQRT: case V_EXP: keep[I.out] = 1; break;
      case V_LOG: case V_RELU: case V_FLOOR: case V_MAX3: case V_ABS: case V_CAP: keep[I.a] = 1; break;
      case V_SDIV: keep[I.b] = keep[I.out] = 1; break;
      case V_SEL: keep[I.c] = 1; break;
      case V_NORM3: keep[I.a] = keep[I.b] = keep[I.c] = keep[I.out] = 1; break;
      default: break;
    }
  }
  std::vector<int> last(S, -1), prod(S, -1);
  for (int q = 0; q < n; ++q) {
    prod[P.code[q].out] = q;
    for (int x : {P.code[q].a, P.code[q].b, P.code[q].c})
      if (x >= 0) last[x] = q;
  }
  // groups of up to kGroupMax operations; a neighbour operation reads its
  // operand at neighbouring cells from memory, so it opens a new group only
  // when that operand is made in the current one
  VPlan R;
  std::vector<int> gid(n), gend;
  for (int q = 0; q < n; ++q) {
    const VInstr& I = P.code[q];
    const bool nb = I.op == V_STEN || I.op == V_MAX3 || I.op == V_MEAN3 || I.op == V_D2 || I.op == V_ROUGH ||
                    I.op == V_PMEAN;
    const bool dep = nb && !R.groups.empty() &&
                     (prod[I.a] >= R.groups.back().first ||
                      (I.op == V_ROUGH && prod[I.b] >= R.groups.back().first));
    // the mask runs in a launch of its own (k_vm_rough): its eight-cell
    // gathers would size the registers of every group's launch
    const bool alone = I.op == V_ROUGH || I.op == V_PMEAN ||
                       (q > 0 && (P.code[q - 1].op == V_ROUGH || P.code[q - 1].op == V_PMEAN));
    if (q == 0 || dep || alone || q - R.groups.back().first == kGroupMax) {
      if (!R.groups.empty()) gend.push_back(q);
      R.groups.push_back({q, 0});
    }
    R.groups.back().count++;
    gid[q] = (int)R.groups.size() - 1;
  }
  gend.push_back(n);
  // a result is stored if a transpose or a later group reads it
  std::vector<char> store(S, 0);
  for (int s = 0; s < 8; ++s) store[s] = 1;
  for (int q = 0; q < n; ++q) {
    const int o = P.code[q].out;
    store[o] = keep[o] || (last[o] >= gend[gid[q]]);
  }
  // value slots for the stored results; a slot is free again at the end of
  // the group of its last reader (a group's first operation may read it at
  // neighbouring cells while other cells of the group already write)
  std::vector<int> vphys(S, -1), freev;
  std::vector<std::vector<int>> release(R.groups.size());
  for (int x = 0; x < 8; ++x) vphys[x] = x;
  R.nval = 8;
  R.steps.resize(n);
  R.fused.resize(n);
  for (int q = 0; q < n; ++q) {
    const VInstr& I = P.code[q];
    if (q == R.groups[gid[q]].first && gid[q] > 0) {
      for (int ph : release[gid[q] - 1]) freev.push_back(ph);
    }
    int ph = -1;
    if (store[I.out]) {
      if (!freev.empty()) {
        ph = freev.back();
        freev.pop_back();
      } else {
        ph = R.nval++;
      }
    }
    vphys[I.out] = ph;
    VInstr F = I;
    F.out = ph;
    F.a = I.a >= 0 ? vphys[I.a] : -1;
    F.b = I.b >= 0 ? vphys[I.b] : -1;
    F.c = I.c >= 0 ? vphys[I.c] : -1;
    R.steps[q].f = F;
    VFused& G = R.fused[q];
    G.f = F;
    const int g0 = R.groups[gid[q]].first;
    auto local = [&](int x) { return (x >= 0 && prod[x] >= g0 && prod[x] < q) ? prod[x] - g0 : -1; };
    G.la = local(I.a);
    G.lb = local(I.b);
    G.lc = local(I.c);
    G.pad = 0;
    int done[3] = {-1, -1, -1}, nd = 0;
    for (int x : {I.a, I.b, I.c}) {
      if (x < 8 || keep[x] || last[x] != q || vphys[x] < 0) continue;
      bool dup = false;
      for (int m = 0; m < nd; ++m) dup |= done[m] == x;
      if (dup) continue;
      done[nd++] = x;
      release[gid[q]].push_back(vphys[x]);
    }
  }
  // the reverse sweep in groups (fills carry no transpose and are skipped);
  // a neighbour transpose reads its output's cotangent at neighbouring cells,
  // so it opens a new group only when a transpose of the current group has
  // added to that cotangent (contrib: position of the last contribution)
  std::vector<int> border, contrib(S, -1);
  for (int q = n - 1; q >= 0; --q) {
    const VInstr& I = P.code[q];
    if (I.op == V_FILL) continue;
    const bool nb = I.op == V_STEN || I.op == V_MAX3 || I.op == V_MEAN3 || I.op == V_D2;
    const bool dep = nb && !R.bgroups.empty() && contrib[I.out] >= R.bgroups.back().first;
    // a plane mean's transpose runs in launches of its own (a plane sum of
    // the cotangent, then its broadcast)
    const bool alone = I.op == V_PMEAN || (!border.empty() && P.code[border.back()].op == V_PMEAN);
    if (R.bgroups.empty() || dep || alone || (int)border.size() - R.bgroups.back().first == kBGroupMax)
      R.bgroups.push_back({(int)border.size(), 0});
    R.bgroups.back().count++;
    for (int x : {I.a, I.b, I.c})
      if (x >= 0) contrib[x] = (int)border.size();
    border.push_back(q);
  }
  // cotangents, allocated in the reverse sweep; a slot is free again at the
  // end of the group of its last use (a group's first transpose may read it
  // at neighbouring cells while other cells of the group already write)
  std::vector<int> cphys(S, -1), freec, pend;
  auto alloc = [&]() {
    if (!freec.empty()) {
      const int c = freec.back();
      freec.pop_back();
      return c;
    }
    return R.ncot++;
  };
  for (int v = 0; v < 8; ++v) R.cout[v] = cphys[P.out[v]] = alloc();
  size_t bg = 0;
  for (size_t u = 0; u < border.size(); ++u) {
    if (bg < R.bgroups.size() && (int)u == R.bgroups[bg].first) {
      for (int c : pend) freec.push_back(c);
      pend.clear();
      ++bg;
    }
    const int q = border[u];
    const VInstr& I = P.code[q];
    VStep& st = R.steps[q];
    st.cout = cphys[I.out];
    st.over = 0;
    int* dst[3] = {&st.ca, &st.cb, &st.cc};
    const int src[3] = {I.a, I.b, I.c};
    for (int m = 0; m < 3; ++m) {
      *dst[m] = -1;
      if (src[m] < 0) continue;
      if (cphys[src[m]] < 0) {
        cphys[src[m]] = alloc();
        st.over |= 1 << m;
      }
      *dst[m] = cphys[src[m]];
    }
    pend.push_back(st.cout);
  }
  for (int v = 0; v < 8; ++v) R.cin[v] = cphys[v];
  for (int q : border) R.bsteps.push_back(R.steps[q]);
  return R;
}

// ---------------------------------------------------------------------------
// Kernels: one thread per cell of the packed boxes (block table as for the
// other whole-box passes).

// Pointwise operations need only the element index o; the neighbour
// operations (stencils, max and mean over three cells) also the cell's
// coordinates, found with 32-bit arithmetic (boxes hold < 2^31 cells).
#define VM_PROLOGUE                                                  \
  const Blk tb_ = tab[blockIdx.x];                                   \
  if ((int)threadIdx.x >= tb_.n) return;                             \
  const BoxDev& bx_ = boxes[tb_.box];                                \
  const unsigned q_ = (unsigned)tb_.start + threadIdx.x;             \
  const long long o = bx_.off + q_;                                  \
  auto coords = [&](int& i, int& j, int& k) {                        \
    const unsigned nx_ = (unsigned)bx_.nx, ny_ = (unsigned)bx_.ny;   \
    const unsigned qx_ = q_ / nx_, qy_ = qx_ / ny_;                   \
    i = (int)(q_ - qx_ * nx_);                                       \
    j = (int)(qx_ - qy_ * ny_);                                      \
    k = (int)qy_;                                                    \
  };

namespace {

// (selects, not a switch: a switch over runtime values becomes a lookup
// table in scratch memory)
__device__ __forceinline__ double geo_of(const BoxDev& b, int geo) {
  double r = 1.0;
  r = geo == G_LX ? b.lv[0] : r;
  r = geo == G_LY ? b.lv[1] : r;
  r = geo == G_LZ ? b.lv[2] : r;
  r = geo == G_H ? b.hmin : r;
  r = geo == G_LXY ? b.le[0] : r;
  r = geo == G_LXZ ? b.le[1] : r;
  r = geo == G_LYZ ? b.le[2] : r;
  r = geo == G_LZF ? b.lv[2] : r;
  r = geo == G_HMIN ? b.hmin : r;
  return r;
}

// The same at plane k: on a stretched z axis the z-dependent factors come
// from the plane's entries of the per-plane table.
template <class T>
__device__ __forceinline__ double geo_at(const BoxDev& b, int geo, const T* zt, int k) {
  if (!b.stretched) return geo_of(b, geo);
  const T* e = zt + b.joff + (long long)k * ZJ_COUNT;
  double r = geo_of(b, geo);
  r = geo == G_LZ ? double(e[ZJ_LZZ]) : r;
  r = geo == G_LXZ ? double(e[ZJ_LXZ]) : r;
  r = geo == G_LYZ ? double(e[ZJ_LYZ]) : r;
  r = geo == G_LZF ? double(e[ZJ_LZF]) : r;
  r = geo == G_H ? double(e[ZJ_H]) : r;
  return r;
}

// Value of a at offset m along axis ax from (i, j, k).
template <class T>
__device__ __forceinline__ T along(const T* a, const Geo<T>& g, int ax, int i, int j, int k, int m) {
  return ax == VX ? a[g.at(i + m, j, k)] : (ax == VY ? a[g.at(i, j + m, k)] : a[g.at(i, j, k + m)]);
}

// Planes of a wall-bounded z axis within this distance of an end take the
// wall forms of the z operators (the tables); the others (and their
// transposes) the periodic pair forms, whose samples then all lie inside.
constexpr int kWallReach = 6;

__device__ __forceinline__ bool wall_z(const BoxDev& b, int ax) { return ax == VZ && b.wall; }
// (on a stretched axis every plane takes the table forms: the Jacobian
// varies from output to output, so the pair forms' transposes do not hold)
__device__ __forceinline__ bool near_end(const BoxDev& b, int k) {
  return b.stretched || k < kWallReach || k >= b.nzt - kWallReach;
}

// The factor of a z derivative at output plane k of a wall-bounded axis:
// the Jacobian of an up (centre) or down (face) output from the per-plane
// table, with the end copy built in (1/dz on a uniform axis).
template <class T>
__device__ __forceinline__ T zjac(const T* zt, const BoxDev& b, int form, int k) {
  return zt[b.joff + (long long)k * ZJ_COUNT + (form ? ZJ_C : ZJ_F)];
}

// Coefficient of input plane p in output plane k of a z operator on a
// wall-bounded axis, before the 1/h of a derivative: fam 0, 1 from the box's
// table (reduced orders at the ends, the end output no stencil reaches
// copying its neighbour's); fam 2 the second-order pair, whose end output
// copies its neighbour's in the same way.
template <class T>
__device__ __forceinline__ T zw_coef(const T* zt, const BoxDev& b, int fam, int form, int k, int p) {
  const int N = b.nzt;
  if (fam == 2) {
    const int c = form ? (k + 1 < N ? k + 1 : N - 1) : (k > 0 ? k : 1);
    return p == c ? T(1) : (p == c - 1 ? T(-1) : T(0));
  }
  const int d = p - k;
  if (d < -3 || d > 3) return T(0);
  const int type = fam == 0 ? (form ? ZT_IUP : ZT_IDN) : (form ? ZT_DUP : ZT_DDN);
  return zt[b.zoff + ((long long)type * N + k) * 7 + d + 3];
}

// The step's reciprocal comes from the box record in global memory: picking
// one of a local Geo's fields by a runtime axis would put Geo in scratch.
template <class T>
__device__ __forceinline__ T sten(const T* a, const Geo<T>& g, const BoxDev& bx, const T* zt, int ax,
                                  int fam, int form, int i, int j, int k) {
  auto at = [&](int m) { return along(a, g, ax, i, j, k, m); };
  const T hinv = T(1.0 / (ax == VX ? bx.dx : (ax == VY ? bx.dy : bx.dz)));
  if (wall_z(bx, ax) && near_end(bx, k)) {
    T acc = T(0);
    const int p0 = k - 3 > 0 ? k - 3 : 0, p1 = k + 3 < bx.nzt - 1 ? k + 3 : bx.nzt - 1;
    for (int p = p0; p <= p1; ++p) acc += zw_coef(zt, bx, fam, form, k, p) * a[g.at(i, j, p)];
    return fam ? acc * (bx.stretched ? zjac(zt, bx, form, k) : hinv) : acc;
  }
  if (fam == 2) return form ? (at(1) - at(0)) * hinv : (at(0) - at(-1)) * hinv;
  if (fam == 0) return form ? op6<0, 1, T>(at, hinv) : op6<0, 0, T>(at, hinv);
  return form ? op6<1, 1, T>(at, hinv) : op6<1, 0, T>(at, hinv);
}

// Transpose of sten at input cell (i, j, k), applied to the cotangent yb of
// its outputs: the opposite stagger (minus it for a derivative), or near
// the ends of a wall axis the gather over the table's columns.
template <class T>
__device__ __forceinline__ T sten_t(const T* yb, const Geo<T>& g, const BoxDev& bx, const T* zt, int ax,
                                    int fam, int form, int i, int j, int k) {
  if (wall_z(bx, ax) && near_end(bx, k)) {
    const T hinv = T(1.0 / bx.dz);
    T acc = T(0);
    const int k0 = k - 3 > 0 ? k - 3 : 0, k1 = k + 3 < bx.nzt - 1 ? k + 3 : bx.nzt - 1;
    if (bx.stretched && fam) {
      for (int q = k0; q <= k1; ++q)
        acc += zw_coef(zt, bx, fam, form, q, k) * zjac(zt, bx, form, q) * yb[g.at(i, j, q)];
      return acc;
    }
    for (int q = k0; q <= k1; ++q) acc += zw_coef(zt, bx, fam, form, q, k) * yb[g.at(i, j, q)];
    return fam ? acc * hinv : acc;
  }
  const T t = sten(yb, g, bx, zt, ax, fam, 1 - form, i, j, k);
  return fam ? -t : t;
}

// Second-order switch: whether cell (i, j, k) is rough (some axis's absolute
// second difference of ln rho or ln e_m above lim), and whether a cell
// touching position `kind` (0 centre, 1 x-edge, 2 y-edge, 3 z-edge of the
// index) is.  On a wall-bounded z axis there is no z second difference on
// the end planes, and a position on the lower end plane touches no cell
// below it.
template <class T>
__device__ __forceinline__ bool rough_cell(const T* lr, const T* le, const Geo<T>& g, int i, int j, int k,
                                           T lim) {
  T m = T(0);
  const bool zd = !g.wall || (k > 0 && k < g.nzt - 1);
  for (int v = 0; v < 2; ++v) {
    const T* a = v ? le : lr;
    const T c = a[g.at(i, j, k)];
    m = fmax(m, fabs(a[g.at(i + 1, j, k)] - T(2) * c + a[g.at(i - 1, j, k)]));
    m = fmax(m, fabs(a[g.at(i, j + 1, k)] - T(2) * c + a[g.at(i, j - 1, k)]));
    if (zd) m = fmax(m, fabs(a[g.at(i, j, k + 1)] - T(2) * c + a[g.at(i, j, k - 1)]));
  }
  return m > lim;
}
template <class T>
__device__ __forceinline__ bool rough_at(const T* lr, const T* le, const Geo<T>& g, int i, int j, int k,
                                         T lim, int kind) {
  const int di = (kind == 2 || kind == 3) ? 1 : 0, dj = (kind == 1 || kind == 3) ? 1 : 0,
            dk = (kind == 1 || kind == 2) ? 1 : 0;
  bool r = false;
  for (int a = 0; a <= dk; ++a) {
    if (g.wall && k - a < 0) continue;
    for (int b = 0; b <= dj; ++b)
      for (int c = 0; c <= di; ++c) r = r || rough_cell(lr, le, g, i - c, j - b, k - a, lim);
  }
  return r;
}

// Value of a at offset m along z from (i, j, k) on a wall-bounded axis, or
// -inf past an end (never chosen by a maximum).
template <class T>
__device__ __forceinline__ T zval_or_ninf(const T* a, const Geo<T>& g, int i, int j, int k, int m) {
  const int q = k + m;
  return (q >= 0 && q < g.nzt) ? a[g.at(i, j, q)] : T(-INFINITY);
}

// Which of (lo, mid, hi) is the first maximal one: 0, 1 or 2.
template <class T> __device__ __forceinline__ int first_max(T lo, T mid, T hi) {
  int s = 0;
  T v = lo;
  if (mid > v) { v = mid; s = 1; }
  if (hi > v) s = 2;
  return s;
}

}  // namespace

// One group of the forward run: the first operation may read neighbouring
// cells from memory; the rest are pointwise, with operands from the group's
// register file (LDS, one column per thread) or from memory.
template <class T>
__global__ __launch_bounds__(kBlock) void k_vm_group(const BoxDev* boxes, const Blk* tab,
                                                     const VFused* __restrict__ code, int first,
                                                     int count, T* base, long long stride,
                                                     const T* __restrict__ zt) {
  __shared__ T regs[kGroupMax * kBlock];
  VM_PROLOGUE
  auto R = [&](int r) -> T& { return regs[r * kBlock + threadIdx.x]; };
  for (int jj = 0; jj < count; ++jj) {
    const VFused G = code[first + jj];
    const VInstr& I = G.f;
    auto opnd = [&](int slot, int loc) -> T { return loc >= 0 ? R(loc) : base[slot * stride + o]; };
    T r;
    switch (I.op) {
      case V_STEN: {
        int i, j, k;
        coords(i, j, k);
        const Geo<T> g(bx_);
        r = sten(base + I.a * stride, g, bx_, zt, I.ax, I.fam, I.form, i, j, k);
        break;
      }
      case V_MAX3: {
        // over the available cells at the ends of a wall axis
        int i, j, k;
        coords(i, j, k);
        const Geo<T> g(bx_);
        const T* a = base + I.a * stride;
        const bool wz = wall_z(bx_, I.ax);
        const T lo = wz ? zval_or_ninf(a, g, i, j, k, -1) : along(a, g, I.ax, i, j, k, -1);
        const T hi = wz ? zval_or_ninf(a, g, i, j, k, 1) : along(a, g, I.ax, i, j, k, 1);
        const T mid = a[o];
        const int s = first_max(lo, mid, hi);
        r = s == 0 ? lo : (s == 1 ? mid : hi);
        break;
      }
      case V_MEAN3: {
        int i, j, k;
        coords(i, j, k);
        const Geo<T> g(bx_);
        const T* a = base + I.a * stride;
        if (wall_z(bx_, I.ax)) {
          // the mean of the available cells, summed in the order k-1, k, k+1
          const bool lo = k > 0, hi = k < bx_.nzt - 1;
          T s = lo ? a[g.at(i, j, k - 1)] + a[o] : a[o];
          if (hi) s = s + a[g.at(i, j, k + 1)];
          r = s / T(1 + (lo ? 1 : 0) + (hi ? 1 : 0));
        } else {
          r = (along(a, g, I.ax, i, j, k, -1) + a[o] + along(a, g, I.ax, i, j, k, 1)) / T(3);
        }
        break;
      }
      case V_D2: {
        int i, j, k;
        coords(i, j, k);
        const Geo<T> g(bx_);
        const T* a = base + I.a * stride;
        // none across the ends of a wall axis
        if (wall_z(bx_, I.ax) && (k == 0 || k == bx_.nzt - 1))
          r = T(0);
        else
          r = along(a, g, I.ax, i, j, k, 1) - T(2) * a[o] + along(a, g, I.ax, i, j, k, -1);
        break;
      }
      case V_ADD: r = opnd(I.a, G.la) + opnd(I.b, G.lb); break;
      case V_SUB: r = opnd(I.a, G.la) - opnd(I.b, G.lb); break;
      case V_MUL: r = opnd(I.a, G.la) * opnd(I.b, G.lb); break;
      case V_DIV: r = opnd(I.a, G.la) / opnd(I.b, G.lb); break;
      case V_SCALE: {
        double gv;
        if (bx_.stretched) {
          int i, j, k;
          coords(i, j, k);
          gv = geo_at(bx_, I.geo, zt, k);
        } else {
          gv = geo_of(bx_, I.geo);
        }
        r = T(I.k * gv) * opnd(I.a, G.la);
        break;
      }
      case V_DIVC: r = opnd(I.a, G.la) / T(I.k); break;
      case V_SQRT: r = sqrt(opnd(I.a, G.la)); break;
      case V_LOG: r = log(opnd(I.a, G.la)); break;
      case V_EXP: r = exp(opnd(I.a, G.la)); break;
      case V_RELU: {
        const T x = opnd(I.a, G.la);
        r = x > T(0) ? x : T(0);
        break;
      }
      case V_FLOOR: {
        const T x = opnd(I.a, G.la);
        r = x > T(I.k) ? x : T(I.k);
        break;
      }
      case V_NORM3: {
        const T x = opnd(I.a, G.la), y = opnd(I.b, G.lb), z = opnd(I.c, G.lc);
        const T s = x * x + y * y + z * z;
        r = s > T(0) ? sqrt(s) : T(0);
        break;
      }
      case V_FILL:
        r = I.geo == G_HINV ? T(I.k / bx_.hmin) : T(I.k * geo_of(bx_, I.geo));
        break;
      case V_ABS: r = fabs(opnd(I.a, G.la)); break;
      case V_SEL: r = opnd(I.c, G.lc) > T(0.5) ? opnd(I.b, G.lb) : opnd(I.a, G.la); break;
      case V_SDIV: {
        const T x = opnd(I.a, G.la), y = opnd(I.b, G.lb);
        r = y > T(0) ? x / y : T(0);
        break;
      }
      case V_CAP: {
        const T x = opnd(I.a, G.la);
        r = x < T(I.k) ? x : T(I.k);
        break;
      }
      default: r = T(0); break;
    }
    R(jj) = r;
    if (I.out >= 0) base[I.out * stride + o] = r;
  }
}

// Transposes.  Each thread owns the cotangents of its own cells, so the
// gathers of the stencil, max and mean transposes need no atomics; the
// pointwise rules update the input cotangents one after the other (an input
// may appear twice, as in a * a: its first contribution overwrites, the
// second adds).  A workgroup takes kBwdCells consecutive block-table entries
// and a thread one cell of each: every transpose first gathers its inputs
// for all of them, so that many loads are in flight per thread.
constexpr int kBwdCells = 4;

template <class T>
__global__ __launch_bounds__(kBlock) void k_vm_bwd(const BoxDev* boxes, const Blk* tab, int nblk,
                                                   const VStep* __restrict__ code, int first,
                                                   int count, const T* base, T* cbase,
                                                   long long stride, const T* __restrict__ zt) {
  constexpr int R = kBwdCells;
  long long o[R];
  unsigned q[R];
  int bi[R];
  bool ok[R];
  bool found = false;
  long long o0 = 0;
  unsigned q0 = 0;
  int b0 = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = (int)blockIdx.x * R + r;
    ok[r] = false;
    bi[r] = 0;
    q[r] = 0;
    o[r] = 0;
    if (e < nblk) {
      const Blk tb = tab[e];
      ok[r] = (int)threadIdx.x < tb.n;
      bi[r] = tb.box;
      q[r] = (unsigned)tb.start + threadIdx.x;
      o[r] = boxes[tb.box].off + q[r];
      if (ok[r] && !found) {
        found = true;
        o0 = o[r];
        q0 = q[r];
        b0 = bi[r];
      }
    }
  }
  if (!found) return;
  // cells past a table entry's end read a valid cell's data and store nothing
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (!ok[r]) {
      o[r] = o0;
      q[r] = q0;
      bi[r] = b0;
    }
  auto coords = [&](int r, int& i, int& j, int& k) {
    const BoxDev& b = boxes[bi[r]];
    const unsigned nx_ = (unsigned)b.nx, ny_ = (unsigned)b.ny;
    const unsigned qx_ = q[r] / nx_, qy_ = qx_ / ny_;
    i = (int)(q[r] - qx_ * nx_);
    j = (int)(qx_ - qy_ * ny_);
    k = (int)qy_;
  };
  for (int jj = 0; jj < count; ++jj) {
    const VStep S = code[first + jj];
    const VInstr& I = S.f;
    const T* a = I.a >= 0 ? base + I.a * stride : nullptr;
    const T* b = I.b >= 0 ? base + I.b * stride : nullptr;
    const T* c = I.c >= 0 ? base + I.c * stride : nullptr;
    T* ca = S.ca >= 0 ? cbase + S.ca * stride : nullptr;
    T* cb = S.cb >= 0 ? cbase + S.cb * stride : nullptr;
    T* cc = S.cc >= 0 ? cbase + S.cc * stride : nullptr;
    const T* yb = cbase + S.cout * stride;
    // the contribution v[r] to dst: overwrite or add, all loads first
    auto put = [&](T* dst, int bit, const T (&v)[R]) {
      T cur[R];
      const bool over = S.over & bit;
#pragma unroll
      for (int r = 0; r < R; ++r) cur[r] = over ? T(0) : dst[o[r]];
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (ok[r]) dst[o[r]] = over ? v[r] : cur[r] + v[r];
    };
    T y[R], v1[R], v2[R], v3[R];
#pragma unroll
    for (int r = 0; r < R; ++r) y[r] = yb[o[r]];
    switch (I.op) {
      case V_STEN: {
        // interpolation: S^T = the opposite stagger; derivative: minus it
#pragma unroll
        for (int r = 0; r < R; ++r) {
          int i, j, k;
          coords(r, i, j, k);
          const Geo<T> g(boxes[bi[r]]);
          v1[r] = sten_t(yb, g, boxes[bi[r]], zt, I.ax, I.fam, I.form, i, j, k);
        }
        put(ca, 1, v1);
        break;
      }
      case V_ADD:
      case V_SUB:
        put(ca, 1, y);
#pragma unroll
        for (int r = 0; r < R; ++r) v2[r] = I.op == V_SUB ? -y[r] : y[r];
        put(cb, 2, v2);
        break;
      case V_MUL:
#pragma unroll
        for (int r = 0; r < R; ++r) {
          v1[r] = y[r] * b[o[r]];
          v2[r] = y[r] * a[o[r]];
        }
        put(ca, 1, v1);
        put(cb, 2, v2);
        break;
      case V_DIV:
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const T vb = b[o[r]], qv = base[I.out * stride + o[r]];
          v1[r] = y[r] / vb;
          v2[r] = -(y[r] * qv / vb);
        }
        put(ca, 1, v1);
        put(cb, 2, v2);
        break;
      case V_SCALE:
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const BoxDev& b = boxes[bi[r]];
          double gv;
          if (b.stretched) {
            int i, j, k;
            coords(r, i, j, k);
            gv = geo_at(b, I.geo, zt, k);
          } else {
            gv = geo_of(b, I.geo);
          }
          v1[r] = T(I.k * gv) * y[r];
        }
        put(ca, 1, v1);
        break;
      case V_DIVC:
#pragma unroll
        for (int r = 0; r < R; ++r) v1[r] = y[r] / T(I.k);
        put(ca, 1, v1);
        break;
      case V_SQRT:
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const T s = base[I.out * stride + o[r]];
          v1[r] = s > T(0) ? y[r] / (T(2) * s) : T(0);
        }
        put(ca, 1, v1);
        break;
      case V_LOG:
#pragma unroll
        for (int r = 0; r < R; ++r) v1[r] = y[r] / a[o[r]];
        put(ca, 1, v1);
        break;
      case V_EXP:
#pragma unroll
        for (int r = 0; r < R; ++r) v1[r] = y[r] * base[I.out * stride + o[r]];
        put(ca, 1, v1);
        break;
      case V_RELU:
#pragma unroll
        for (int r = 0; r < R; ++r) v1[r] = a[o[r]] > T(0) ? y[r] : T(0);
        put(ca, 1, v1);
        break;
      case V_FLOOR:
#pragma unroll
        for (int r = 0; r < R; ++r) v1[r] = a[o[r]] > T(I.k) ? y[r] : T(0);
        put(ca, 1, v1);
        break;
      case V_NORM3:
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const T nrm = base[I.out * stride + o[r]];
          const T w = nrm > T(0) ? y[r] / nrm : T(0);
          v1[r] = w * a[o[r]];
          v2[r] = w * b[o[r]];
          v3[r] = w * c[o[r]];
        }
        put(ca, 1, v1);
        put(cb, 2, v2);
        put(cc, 4, v3);
        break;
      case V_MAX3:
        // cell (i) is the hi neighbour of i-1, the middle of i, the lo of i+1
#pragma unroll
        for (int r = 0; r < R; ++r) {
          int i, j, k;
          coords(r, i, j, k);
          const Geo<T> g(boxes[bi[r]]);
          // on a wall axis: cells past an end are -inf, outputs past an end absent
          const bool wz = wall_z(boxes[bi[r]], I.ax);
          auto v = [&](int m) { return wz ? zval_or_ninf(a, g, i, j, k, m) : along(a, g, I.ax, i, j, k, m); };
          auto w = [&](int m) { return along(yb, g, I.ax, i, j, k, m); };
          const T vm2 = v(-2), vm1 = v(-1), v0 = a[o[r]], vp1 = v(1), vp2 = v(2);
          const bool has_lo = !wz || k > 0, has_hi = !wz || k < g.nzt - 1;
          T sum = T(0);
          if (has_lo && first_max(vm2, vm1, v0) == 2) sum += w(-1);
          if (first_max(vm1, v0, vp1) == 1) sum += y[r];
          if (has_hi && first_max(v0, vp1, vp2) == 0) sum += w(1);
          v1[r] = sum;
        }
        put(ca, 1, v1);
        break;
      case V_MEAN3:
#pragma unroll
        for (int r = 0; r < R; ++r) {
          int i, j, k;
          coords(r, i, j, k);
          const Geo<T> g(boxes[bi[r]]);
          if (wall_z(boxes[bi[r]], I.ax)) {
            // output q averages over 2 cells at an end of the axis, else 3
            const int N = g.nzt;
            auto cnt = [&](int q) { return T(q == 0 || q == N - 1 ? 2 : 3); };
            T s = y[r] / cnt(k);
            if (k > 0) s += yb[g.at(i, j, k - 1)] / cnt(k - 1);
            if (k < N - 1) s += yb[g.at(i, j, k + 1)] / cnt(k + 1);
            v1[r] = s;
          } else {
            v1[r] = (along(yb, g, I.ax, i, j, k, -1) + y[r] + along(yb, g, I.ax, i, j, k, 1)) / T(3);
          }
        }
        put(ca, 1, v1);
        break;
      case V_D2:   // symmetric on a periodic axis
#pragma unroll
        for (int r = 0; r < R; ++r) {
          int i, j, k;
          coords(r, i, j, k);
          const Geo<T> g(boxes[bi[r]]);
          if (wall_z(boxes[bi[r]], I.ax)) {
            // outputs 1 .. N-2 only
            const int N = g.nzt;
            T s = (k >= 1 && k <= N - 2) ? T(-2) * y[r] : T(0);
            if (k - 1 >= 1) s += yb[g.at(i, j, k - 1)];
            if (k + 1 <= N - 2) s += yb[g.at(i, j, k + 1)];
            v1[r] = s;
          } else {
            v1[r] = along(yb, g, I.ax, i, j, k, 1) - T(2) * y[r] + along(yb, g, I.ax, i, j, k, -1);
          }
        }
        put(ca, 1, v1);
        break;
      case V_ABS:
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const T x = a[o[r]];
          v1[r] = x > T(0) ? y[r] : (x < T(0) ? -y[r] : T(0));
        }
        put(ca, 1, v1);
        break;
      case V_SDIV:
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const T vb = b[o[r]], qv = base[I.out * stride + o[r]];
          v1[r] = vb > T(0) ? y[r] / vb : T(0);
          v2[r] = vb > T(0) ? -(y[r] * qv / vb) : T(0);
        }
        put(ca, 1, v1);
        put(cb, 2, v2);
        break;
      case V_CAP:
#pragma unroll
        for (int r = 0; r < R; ++r) v1[r] = a[o[r]] < T(I.k) ? y[r] : T(0);
        put(ca, 1, v1);
        break;
      case V_ROUGH:   // a mask: no derivative
#pragma unroll
        for (int r = 0; r < R; ++r) v1[r] = T(0);
        put(ca, 1, v1);
        put(cb, 2, v1);
        break;
      case V_SEL:
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const bool m = c[o[r]] > T(0.5);
          v1[r] = m ? T(0) : y[r];
          v2[r] = m ? y[r] : T(0);
          v3[r] = T(0);
        }
        put(ca, 1, v1);
        put(cb, 2, v2);
        put(cc, 4, v3);
        break;
      default: break;
    }
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_axpby8(const BoxDev* boxes, const Blk* tab, P8<T> y,
                                                   CP8<T> x, T a, T b) {
  VM_PROLOGUE
  (void)coords;
  for (int v = 0; v < 8; ++v) {
    const T xv = x.p[0] ? x.p[v][o] : T(0);
    y.p[v][o] = (a == T(0) ? T(0) : a * y.p[v][o]) + b * xv;
  }
}

// The second-order switch's mask (V_ROUGH), alone in its group: both
// operands and the result in memory.
template <class T>
__global__ __launch_bounds__(kBlock) void k_vm_rough(const BoxDev* boxes, const Blk* tab,
                                                     const VFused* __restrict__ code, int at, T* base,
                                                     long long stride) {
  VM_PROLOGUE
  const VInstr I = code[at].f;
  int i, j, k;
  coords(i, j, k);
  const Geo<T> g(bx_);
  base[I.out * stride + o] =
      rough_at(base + I.a * stride, base + I.b * stride, g, i, j, k, T(I.k), I.ax) ? T(1) : T(0);
}

// V_PMEAN: the mean of src over each z plane of every box, in float64 and a
// fixed order (one workgroup per plane), then its broadcast over the plane
// into dst (overwriting, or added with over = 0).
constexpr int kPlaneBlock = 256;
template <class T>
__global__ __launch_bounds__(kPlaneBlock) void k_vm_psum(const BoxDev* __restrict__ boxes, int nbox,
                                                        const T* __restrict__ src, double* __restrict__ pm) {
  __shared__ double sh[kPlaneBlock];
  const int P = (int)blockIdx.x;
  int bi = 0;
  while (bi + 1 < nbox && boxes[bi + 1].poff <= P) ++bi;
  const BoxDev& b = boxes[bi];
  const int n = b.nx * b.ny;
  const T* __restrict__ s = src + b.off + (long long)(P - b.poff) * n;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kPlaneBlock) acc += (double)s[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kPlaneBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) pm[P] = sh[0] / (double)n;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_vm_pbcast(const BoxDev* boxes, const Blk* tab,
                                                      const double* __restrict__ pm, T* dst, int over) {
  VM_PROLOGUE
  int i, j, k;
  coords(i, j, k);
  const T v = T(pm[bx_.poff + k]);
  dst[o] = over ? v : dst[o] + v;
}

template <class T>
static void vm_pmean(const VLaunch& L, const T* src, T* dst, int over) {
  hipLaunchKernelGGL(k_vm_psum<T>, dim3(L.nplanes), dim3(kPlaneBlock), 0, L.stream, L.boxes, L.nbox, src, L.pm);
  hipLaunchKernelGGL(k_vm_pbcast<T>, dim3(L.nblk), dim3(kBlock), 0, L.stream, L.boxes, L.tab,
                     (const double*)L.pm, dst, over);
}

// ---------------------------------------------------------------------------
// Transpose of the closed-wall ghost fill (Section 10 "Closed"), linearised
// at the filled state s.  The fill sets, on ghost plane k at distance d from
// the wall, from interior planes a0 (next to the wall) and a1:
//   rho_k = exp(L_r), L_r = (1 + d) ln rho_a0 - d ln rho_a1,
//   e_k = rho_k exp(L_m), L_m the same of ln(e / rho),
//   p_x,k = X_k p_x,m / X_m with X = xdn(rho) on planes k and m (the mirror
//   across the wall; p_y with ydn), B_x,k = -B_x,m, B_y,k = -B_y,m,
//   p_z and B_z beyond the wall face mirrored (- and +), p_z = 0 on both
//   wall faces.
// One thread per ghost cell of one side (lower side 0, upper 1; the sides
// run apart, since their mirror planes can meet in a shallow box), in three
// launches: (1) the cotangents of X_k and X_m of each ghost p_x, p_y cell
// into tmp 0..3 and the mirror contributions to p_x, p_y, B and p_z; (2) the
// cotangent of the ghost density (through X_k and e_k), of L_r and L_m into
// tmp 4, 5, and that of the mirror density through X_m; (3) per column the
// sums over the side's ghost planes into rho and e at a0 and a1, and the
// ghost cotangents cleared.
namespace {
struct GhostCell {
  int i, j, k, m, d, a0, a1;
  bool lower;
};
__device__ __forceinline__ bool ghost_cell(const BoxDev& b, const Blk& t, int side, GhostCell& c) {
  long long q = t.start + threadIdx.x;   // over nx * ny * (2 ngz)
  c.i = (int)(q % b.nx);
  q /= b.nx;
  c.j = (int)(q % b.ny);
  const int s = (int)(q / b.ny);
  c.lower = s < b.ngz;
  if (c.lower != (side == 0)) return false;
  c.k = c.lower ? s : b.g1 + (s - b.ngz);
  c.d = c.lower ? b.g0 - c.k : c.k - b.g1 + 1;
  c.m = c.lower ? 2 * b.g0 - 1 - c.k : 2 * b.g1 - 1 - c.k;
  c.a0 = c.lower ? b.g0 : b.g1 - 1;
  c.a1 = c.lower ? b.g0 + 1 : b.g1 - 2;
  return true;
}
}  // namespace

template <class T>
__global__ __launch_bounds__(kBlock) void k_fill_vjp1(const BoxDev* boxes, const Blk* gtab, int side, CP8<T> s,
                                                      P8<T> g, T* t0, T* t1, T* t2, T* t3) {
  const Blk t = gtab[blockIdx.x];
  if ((int)threadIdx.x >= t.n) return;
  const BoxDev& b = boxes[t.box];
  GhostCell c;
  if (!ghost_cell(b, t, side, c)) return;
  const Geo<T> G(b);
  const int i = c.i, j = c.j, k = c.k, m = c.m;
  const long long o = G.at(i, j, k), om = G.at(i, j, m);
  const T* rho = s.p[0];
  const T xk = op6<0, 0, T>([&](int l) { return rho[G.at(i + l, j, k)]; }, T(0));
  const T xm = op6<0, 0, T>([&](int l) { return rho[G.at(i + l, j, m)]; }, T(0));
  const T yk = op6<0, 0, T>([&](int l) { return rho[G.at(i, j + l, k)]; }, T(0));
  const T ym = op6<0, 0, T>([&](int l) { return rho[G.at(i, j + l, m)]; }, T(0));
  const T gpx = g.p[1][o], gpy = g.p[2][o];
  const T pxm = s.p[1][om], pym = s.p[2][om];
  t0[o] = gpx * (pxm / xm);
  t1[o] = gpy * (pym / ym);
  t2[o] = -(gpx * (xk * pxm / xm) / xm);
  t3[o] = -(gpy * (yk * pym / ym) / ym);
  g.p[1][om] += gpx * (xk / xm);
  g.p[2][om] += gpy * (yk / ym);
  g.p[5][om] -= g.p[5][o];
  g.p[6][om] -= g.p[6][o];
  // z-faces beyond the wall face mirror the faces inside it
  if (c.lower || k != b.g1) {
    const long long of = G.at(i, j, c.lower ? 2 * b.g0 - k : 2 * b.g1 - k);
    g.p[3][of] -= g.p[3][o];
    g.p[7][of] += g.p[7][o];
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_fill_vjp2(const BoxDev* boxes, const Blk* gtab, int side, CP8<T> s,
                                                      P8<T> g, const T* t0, const T* t1, const T* t2,
                                                      const T* t3, T* t4, T* t5) {
  const Blk t = gtab[blockIdx.x];
  if ((int)threadIdx.x >= t.n) return;
  const BoxDev& b = boxes[t.box];
  GhostCell c;
  if (!ghost_cell(b, t, side, c)) return;
  const Geo<T> G(b);
  const int i = c.i, j = c.j, k = c.k;
  const long long o = G.at(i, j, k), om = G.at(i, j, c.m);
  // transposes of xdn, ydn on a periodic axis: xup, yup
  const T rk = g.p[0][o] + op6<0, 1, T>([&](int l) { return t0[G.at(i + l, j, k)]; }, T(0)) +
               op6<0, 1, T>([&](int l) { return t1[G.at(i, j + l, k)]; }, T(0));
  const T rn = s.p[0][o], en = s.p[4][o], ge = g.p[4][o];
  t4[o] = (rk + ge * (en / rn)) * rn;
  t5[o] = ge * en;
  g.p[0][om] += op6<0, 1, T>([&](int l) { return t2[G.at(i + l, j, k)]; }, T(0)) +
                op6<0, 1, T>([&](int l) { return t3[G.at(i, j + l, k)]; }, T(0));
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_fill_vjp3(const BoxDev* boxes, const Blk* gtab, int side, CP8<T> s,
                                                      P8<T> g, const T* t4, const T* t5) {
  const Blk t = gtab[blockIdx.x];
  if ((int)threadIdx.x >= t.n) return;
  const BoxDev& b = boxes[t.box];
  GhostCell c;
  if (!ghost_cell(b, t, side, c)) return;
  const Geo<T> G(b);
  const int i = c.i, j = c.j, k = c.k;
  const long long o = G.at(i, j, k);
  if (c.d == 1) {
    // L_r and L_m of every ghost plane of this side, into ln rho, ln e_m at a0, a1
    T lr0 = T(0), lr1 = T(0), lm0 = T(0), lm1 = T(0);
    for (int dd = 1; dd <= b.ngz; ++dd) {
      const long long oq = G.at(i, j, c.lower ? b.g0 - dd : b.g1 - 1 + dd);
      lr0 += T(1 + dd) * t4[oq];
      lr1 -= T(dd) * t4[oq];
      lm0 += T(1 + dd) * t5[oq];
      lm1 -= T(dd) * t5[oq];
    }
    const long long o0 = G.at(i, j, c.a0), o1 = G.at(i, j, c.a1);
    // ln e_m = ln e - ln rho
    g.p[0][o0] += (lr0 - lm0) / s.p[0][o0];
    g.p[4][o0] += lm0 / s.p[4][o0];
    g.p[0][o1] += (lr1 - lm1) / s.p[0][o1];
    g.p[4][o1] += lm1 / s.p[4][o1];
    if (c.lower) g.p[3][G.at(i, j, b.g0)] = T(0);   // p_z on the lower wall face
  }
  // the fill overwrites every ghost value except B_z on the upper wall face
#pragma unroll
  for (int v = 0; v < 8; ++v)
    if (!(v == 7 && k == b.g1)) g.p[v][o] = T(0);
}

// Zero where the right-hand side is zeroed on a wall box: the ghost planes
// of centred fields, p_z outside the open interior faces, B_z outside the
// faces from wall to wall.
template <class T>
__global__ __launch_bounds__(kBlock) void k_wall_mask8(const BoxDev* boxes, const Blk* tab, P8<T> y) {
  VM_PROLOGUE
  if (!bx_.wall) return;
  int i, j, k;
  coords(i, j, k);
  (void)i;
  (void)j;
  const bool cen = k >= bx_.g0 && k < bx_.g1;
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const bool keep = v == 3 ? (k > bx_.g0 && k < bx_.g1) : (v == 7 ? (k >= bx_.g0 && k <= bx_.g1) : cen);
    if (!keep) y.p[v][o] = T(0);
  }
}

template <class T> void vm_fill_vjp(const VLaunch& L, CP8<T> s, P8<T> g, T* tmp, long long stride) {
  if (L.nghost_blk == 0) return;
  T* t[6];
  for (int q = 0; q < 6; ++q) t[q] = tmp + (long long)q * stride;
  for (int side = 0; side < 2; ++side) {
    hipLaunchKernelGGL(k_fill_vjp1<T>, dim3(L.nghost_blk), dim3(kBlock), 0, L.stream, L.boxes, L.gtab, side, s,
                       g, t[0], t[1], t[2], t[3]);
    hipLaunchKernelGGL(k_fill_vjp2<T>, dim3(L.nghost_blk), dim3(kBlock), 0, L.stream, L.boxes, L.gtab, side, s,
                       g, (const T*)t[0], (const T*)t[1], (const T*)t[2], (const T*)t[3], t[4], t[5]);
    hipLaunchKernelGGL(k_fill_vjp3<T>, dim3(L.nghost_blk), dim3(kBlock), 0, L.stream, L.boxes, L.gtab, side, s,
                       g, (const T*)t[4], (const T*)t[5]);
  }
}

template <class T> void vm_wall_mask(const VLaunch& L, P8<T> g) {
  hipLaunchKernelGGL(k_wall_mask8<T>, dim3(L.nblk), dim3(kBlock), 0, L.stream, L.boxes, L.tab, g);
}

template <class T>
void vm_forward(const VLaunch& L, const VPlan& P, const VFused* d_fused, T* base, long long stride) {
  for (const VGroup& G : P.groups) {
    const VInstr& I = P.fused[G.first].f;
    if (I.op == V_ROUGH)
      hipLaunchKernelGGL(k_vm_rough<T>, dim3(L.nblk), dim3(kBlock), 0, L.stream, L.boxes, L.tab, d_fused,
                         G.first, base, stride);
    else if (I.op == V_PMEAN)
      vm_pmean<T>(L, base + I.a * stride, base + I.out * stride, 1);
    else
      hipLaunchKernelGGL(k_vm_group<T>, dim3(L.nblk), dim3(kBlock), 0, L.stream, L.boxes, L.tab, d_fused,
                         G.first, G.count, base, stride, (const T*)L.ztab);
  }
}

template <class T>
void vm_backward(const VLaunch& L, const VPlan& P, const VStep* d_bsteps, const T* base, T* cbase,
                 long long stride) {
  const int grid = (L.nblk + kBwdCells - 1) / kBwdCells;
  for (const VGroup& G : P.bgroups) {
    const VStep& S = P.bsteps[G.first];
    if (S.f.op == V_PMEAN) {
      vm_pmean<T>(L, (const T*)(cbase + S.cout * stride), cbase + S.ca * stride, S.over & 1);
      continue;
    }
    hipLaunchKernelGGL(k_vm_bwd<T>, dim3(grid), dim3(kBlock), 0, L.stream, L.boxes, L.tab, L.nblk,
                       d_bsteps, G.first, G.count, base, cbase, stride, (const T*)L.ztab);
  }
}

template <class T> void vm_axpby8(const VLaunch& L, P8<T> y, CP8<T> x, double a, double b) {
  hipLaunchKernelGGL(k_axpby8<T>, dim3(L.nblk), dim3(kBlock), 0, L.stream, L.boxes, L.tab, y, x, T(a),
                     T(b));
}

template void vm_forward<float>(const VLaunch&, const VPlan&, const VFused*, float*, long long);
template void vm_forward<double>(const VLaunch&, const VPlan&, const VFused*, double*, long long);
template void vm_backward<float>(const VLaunch&, const VPlan&, const VStep*, const float*, float*,
                                 long long);
template void vm_backward<double>(const VLaunch&, const VPlan&, const VStep*, const double*, double*,
                                  long long);
template void vm_axpby8<float>(const VLaunch&, P8<float>, CP8<float>, double, double);
template void vm_axpby8<double>(const VLaunch&, P8<double>, CP8<double>, double, double);
template void vm_fill_vjp<float>(const VLaunch&, CP8<float>, P8<float>, float*, long long);
template void vm_fill_vjp<double>(const VLaunch&, CP8<double>, P8<double>, double*, long long);
template void vm_wall_mask<float>(const VLaunch&, P8<float>);
template void vm_wall_mask<double>(const VLaunch&, P8<double>);

}  // namespace smhd
