// z-marching kernels of one RK stage (the production forward path).
//
// Five passes per stage, in eight launches over all (box, tile, z-range)
// work items (Q in two: edges, then z-face and centre terms; F in three, one
// per field group):
//   A1  face velocity u_z, div u, and the speed-like viscosity
//       nu1|u| + nu3(c_s + c_A) + nu2 h max(0, -div u)         (eq. RMnu)
//   A2  maximum over three cells then three-cell mean, floor, ln  (Section 6.1.1)
//   Q   quantities on x- and y-directed cell edges (stress, E, Lorentz
//       products, heating; eqs. itv, nuij, ohm, vdiss) and the z-face /
//       centre terms that need z derivatives of z-stencil results (Gzz, Hz)
//   P   quantities on z-directed edges and the x/y parts of the centre and
//       face terms (only x/y stencils)
//   F   all divergences (eqs. mass, mom, ien, indu), gravity, wall masking
//       and the fused RK stage update (eqs. ddt, tupdate)
// Stage-1 launches of A1 / A2 also leave per-item maxima for the Courant
// time step (eq. courantcond), which k_dt folds into a device-resident dt.
#include <algorithm>
#include <map>
#include <utility>
#include <mutex>

#include "mhd_zmarch.hpp"
#include "mhd_zstage.hpp"

namespace smhd {

// ---------------------------------------------------------------------------
// A1: u_z = p_z / zdn(rho); div u; speed-like viscosity nu_s.
// Front plane r: x/y stencils of plane r go through LDS, their results wait
// in short per-thread queues; u_z (plane r-2) and the z stencils (plane r-5)
// come from register windows.
//
// RED (the reduction instantiation of mhd_reductions): also accumulates, in
// float64 over the item's interior cells, the totals of the state, div B and
// the maxima, the wave speed c_s + c_A + |u_perp| and the rate
// max(|d ln rho/dt|, |d ln e_m/dt|) with the cells that set them, into
// red[item].
// SMAG (with T_SMAG): also writes what pass S needs for the Smagorinsky
// viscosity into the workspace of pass Q (free until then): the centred
// velocities aup(u_a) and the diagonal strain ddaup(u_a).
template <class T, int TX, int TY, bool PERS, bool RED = false, bool SMAG = false>
__global__ __launch_bounds__(TX * TY) void zA1(const BoxDev* __restrict__ boxes,
                                               const ZItem* __restrict__ items, int nitems, const T* __restrict__ ztab,
                                               int* __restrict__ queue,
                                               CP8<T> f, Phys<T> ph, ZWork<T> ws,
                                               CPart* __restrict__ cpart,
                                               CP8<T> dfdt = CP8<T>{}, RedItem* __restrict__ red = nullptr) {
  T* __restrict__ nus_out = ws.arr(WS_NUS);
  T* __restrict__ D_out = ws.arr(WS_D);
  T* __restrict__ divb_out = ws.arr(WS_DIVB);
  const bool divb = ph.terms & T_DIVB;
  constexpr int NW = TX * TY / 64;
  __shared__ double sredw[RED ? NW * 15 : 1];
  __shared__ long long sredl[RED ? NW * 4 : 1];
  T* __restrict__ uz_out = ws.arr(WS_UZ);
  using PR = Plane<TX, TY, 5>;
  using PP = Plane<TX, TY, 3>;
  constexpr int NT = TX * TY;
  __shared__ T sR[PR::NP];
  __shared__ T sPX[PP::NP], sPY[PP::NP], sBX[PP::NP], sBY[PP::NP];
  // face velocities of the plane, computed once per face: u_x at x-offsets
  // -2..3 of the own rows, u_y at y-offsets -2..3 of the own columns
  __shared__ T sUX[PP::NP], sUY[PP::NP];
  __shared__ double sred[TX * TY];
  ZLOOP_BEGIN
  PlaneIdx<TX, TY, 5> i5;
  PlaneIdx<TX, TY, 3> i3;
  i5.init(b, it.x0, it.y0);
  i3.init(b, it.x0, it.y0);
  T wR[6] = {}, wUZ[6] = {}, wBZ[8] = {}, fPZ[3] = {}, fE[6] = {};
  T fUBX[6] = {}, fUBY[6] = {}, fBBX[6] = {}, fBBY[6] = {}, fDXY[6] = {}, fDXB[6] = {};
  double cmax = 0.0;
  // reduction accumulators (RED): sums, maxima, (max, cell) pairs, counts
  double rs[8] = {}, rdiv = 0.0, rbm = 0.0, rum = 0.0, rc = 0.0, rrate = 0.0;
  long long rca = 0x7fffffffffffffffLL, rra = 0x7fffffffffffffffLL, rnf = 0, rnp = 0;
  auto packed = [&](int k_) { return b.off + ((long long)k_ * b.ny + gy) * b.nx + gx; };
  // rho (halo 5) of plane r is fetched into registers one iteration ahead;
  // the last fetch repeats the last valid plane
  constexpr int N5 = PlaneIdx<TX, TY, 5>::NPER;
  static_assert(N5 * NT == PR::NP, "plane padding");
  const int rfirst = wall ? max(it.z0 - 5, 0) : it.z0 - 5;
  const int rlast = wall ? min(it.z1 + 4, N - 1) : it.z1 + 4;
  T gR5[N5];
  auto fetch = [&](int r_) {
    const long long pk = b.off + (long long)kk(r_) * pstride;
#pragma unroll
    for (int i = 0; i < N5; ++i) gR5[i] = f.p[0][pk + i5.off[i]];
  };
  fetch(rfirst);
  for (int r = it.z0 - 5; r <= it.z1 + 4; ++r) {
    T rr = T(0), pz = T(0), e = T(0), bz = T(0);
    T ubx = T(0), uby = T(0), bbx = T(0), bby = T(0), dxy = T(0), dxb = T(0);
    if (valid(r)) {
      const int k = kk(r);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < N5; ++i) sR[(int)threadIdx.x + i * NT] = gR5[i];
      load_plane(sPX, f.p[1], b, i3, k);
      load_plane(sPY, f.p[2], b, i3, k);
      load_plane(sBX, f.p[5], b, i3, k);
      load_plane(sBY, f.p[6], b, i3, k);
      // the own column's values, in flight with the planes
      const long long o = col(r);
      pz = f.p[3][o];
      e = f.p[4][o];
      bz = f.p[7][o];
      fetch(r < rlast ? r + 1 : r);
      __syncthreads();
      rr = sR[PR::at(tx, ty)];
      // u_x = p_x / xdn(rho) on x-faces -2..3 of the own rows and u_y on
      // y-faces -2..3 of the own columns, one face per thread and pass
      for (int t = threadIdx.x; t < PP::N; t += NT) {
        const int yy = t / PP::W, xx = t - yy * PP::W;
        const int x = xx - 3, y = yy - 3;
        if (y >= 0 && y < TY && x >= -2)
          sUX[t] = sPX[t] / op6<0, 0, T>([&](int a) { return sR[PR::at(x + a, y)]; }, T(0));
        if (x >= 0 && x < TX && y >= -2)
          sUY[t] = sPY[t] / op6<0, 0, T>([&](int a) { return sR[PR::at(x, y + a)]; }, T(0));
      }
      __syncthreads();
      ubx = op6<0, 1, T>([&](int m) { return sUX[PP::at(tx + m, ty)]; }, T(0));
      uby = op6<0, 1, T>([&](int m) { return sUY[PP::at(tx, ty + m)]; }, T(0));
      dxy = op6<1, 1, T>([&](int m) { return sUX[PP::at(tx + m, ty)]; }, g.hxi) +
            op6<1, 1, T>([&](int m) { return sUY[PP::at(tx, ty + m)]; }, g.hyi);
      bbx = op6<0, 1, T>([&](int m) { return sBX[PP::at(tx + m, ty)]; }, T(0));
      bby = op6<0, 1, T>([&](int m) { return sBY[PP::at(tx, ty + m)]; }, T(0));
      if (SMAG && own && r >= it.z0 && r < it.z1) {
        const long long o = col(r);
        ws.q(3)[o] = op6<1, 1, T>([&](int m) { return sUX[PP::at(tx + m, ty)]; }, g.hxi);
        ws.q(4)[o] = op6<1, 1, T>([&](int m) { return sUY[PP::at(tx, ty + m)]; }, g.hyi);
      }
      // x and y parts of div B at the centre (the div B diffusion)
      if (divb || RED)
        dxb = op6<1, 1, T>([&](int m) { return sBX[PP::at(tx + m, ty)]; }, g.hxi) +
              op6<1, 1, T>([&](int m) { return sBY[PP::at(tx, ty + m)]; }, g.hyi);
      // totals over the own cell of an interior plane (faces at the lower side)
      if (RED && own && r >= it.z0 && r < it.z1 && interior(r)) {
        const double rd = rr, pxd = sPX[PP::at(tx, ty)], pyd = sPY[PP::at(tx, ty)], pzd = pz;
        const double ed = e, bxd = sBX[PP::at(tx, ty)], byd = sBY[PP::at(tx, ty)], bzd = bz;
        const double uxd = sUX[PP::at(tx, ty)], uyd = sUY[PP::at(tx, ty)];
        const double v8[8] = {rd, pxd, pyd, pzd, ed, bxd, byd, bzd};
        for (int v = 0; v < 8; ++v) rnf += isfinite(v8[v]) ? 0 : 1;
        if (!(rd > 0.0) || !(ed > 0.0)) ++rnp;
        // the cell's volume relative to dx dy dz (a stretched z axis)
        const double wz = b.stretched ? double(zj(r, ZJ_DZC)) / b.dz : 1.0;
        rs[0] += rd * wz;
        rs[1] += pxd * wz;
        rs[2] += pyd * wz;
        rs[3] += pzd * wz;
        rs[4] += 0.5 * (pxd * uxd + pyd * uyd) * wz;
        rs[5] += (bxd * bxd + byd * byd + bzd * bzd) * wz;
        rs[6] += ed * wz;
        rbm = fmax(rbm, fmax(fabs(bxd), fmax(fabs(byd), fabs(bzd))));
        rum = fmax(rum, fmax(fabs(uxd), fabs(uyd)));
        if (dfdt.p[0]) {
          const long long o = col(r);
          const double dr = (double)dfdt.p[0][o] / rd;
          const double dem = (double)dfdt.p[4][o] / ed - dr;
          const double rate = fmax(fabs(dr), fabs(dem));
          if (rate > rrate) {
            rrate = rate;
            rra = packed(r);
          }
        }
      }
    }
    push(wR, rr);
    push(fPZ, pz);
    push(fE, e);
    push(wBZ, bz);
    push(fUBX, ubx);
    push(fUBY, uby);
    push(fBBX, bbx);
    push(fBBY, bby);
    push(fDXY, dxy);
    push(fDXB, dxb);
    // u_z on the face of plane q1 = r - 2 (wR slot 3 holds plane q1)
    const int q1 = r - 2;
    T uzq = T(0);
    if (valid(q1)) {
      const T zr = zwin<0, 0, 6, 3>(wR, q1, wall, N, T(0), zt);
      uzq = fPZ[0] / zr;
      if (own && q1 >= it.z0 && q1 < it.z1) uz_out[col(q1)] = uzq;
      if (RED && own && q1 >= it.z0 && q1 < it.z1 && interior(q1)) {
        rs[4] += 0.5 * (double)fPZ[0] * (double)uzq * (b.stretched ? double(zj(q1, ZJ_DZC)) / b.dz : 1.0);
        rum = fmax(rum, fabs((double)uzq));
      }
    }
    push(wUZ, uzq);                       // wUZ slot m = plane r-7+m
    // centre quantities of plane q = r - 5
    const int q = r - 5;
    if (valid(q) && q >= it.z0 && q < it.z1) {
      const T ubz = zwin<0, 1, 6, 2>(wUZ, q, wall, N, T(0), zt);
      const T dzz = zwin<1, 1, 6, 2>(wUZ, q, wall, N, zj(q, ZJ_C), zt);
      const T bbz = zwin<0, 1, 8, 2>(wBZ, q, wall, N, T(0), zt);
      const T rq = wR[0], eq = fE[0];
      const T D = fDXY[0] + dzz;
      const T P = ph.gamma1 * eq;
      const T cs = sqrt(ph.gamma * P / rq);
      const T bb = norm3(fBBX[0], fBBY[0], bbz);
      const T ca = bb / sqrt(ph.mu * rq);
      T nus;
      if (ph.nu_const > T(0)) {
        nus = ph.nu_const / g.h;
      } else {
        const T relu = -D > T(0) ? -D : T(0);
        nus = ph.nu1 * norm3(fUBX[0], fUBY[0], ubz) + ph.nu3 * (cs + ca) + ph.nu2 * zj(q, ZJ_H) * relu;
      }
      if (own) {
        const long long o = col(q);
        nus_out[o] = nus;
        D_out[o] = D;
        if (SMAG) {
          ws.q(0)[o] = fUBX[0];
          ws.q(1)[o] = fUBY[0];
          ws.q(2)[o] = ubz;
          ws.q(5)[o] = dzz;
        }
        if (divb) divb_out[o] = fDXB[0] + zwin<1, 1, 8, 2>(wBZ, q, wall, N, zj(q, ZJ_C), zt);
        if ((cpart || RED) && interior(q)) {
          const double ux_ = fUBX[0], uy_ = fUBY[0], uz_ = ubz;
          const double bx_ = fBBX[0], by_ = fBBY[0], bz_ = bbz, bbd = bb;
          const double udotb = bbd > 0.0 ? (ux_ * bx_ + uy_ * by_ + uz_ * bz_) / bbd : 0.0;
          const double uu = ux_ * ux_ + uy_ * uy_ + uz_ * uz_;
          const double up = sqrt(fmax(uu - udotb * udotb, 0.0));
          const double c_ = (double)cs + (double)ca + up;
          cmax = fmax(cmax, c_);
          if (RED) {
            if (c_ > rc) {
              rc = c_;
              rca = packed(q);
            }
            const double db = (double)fDXB[0] + (double)zwin<1, 1, 8, 2>(wBZ, q, wall, N, zj(q, ZJ_C), zt);
            rs[7] += db * db;
            rdiv = fmax(rdiv, fabs(db));
          }
        }
      }
    }
  }
  if (cpart) {
    const double m = block_max<TX * TY>(cmax, sred);
    if (threadIdx.x == 0) cpart[item_].cmax = m;
  }
  if constexpr (RED) {
    // wavefront reductions, then the waves in order in thread 0
    const int w = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
    double* sw = sredw + w * 15;
    long long* sl = sredl + w * 4;
    for (int q = 0; q < 8; ++q) rs[q] = wave_sum(rs[q]);
    rdiv = wave_max(rdiv);
    rbm = wave_max(rbm);
    rum = wave_max(rum);
    wave_maxarg(rc, rca);
    wave_maxarg(rrate, rra);
    const long long nf = wave_isum(rnf), np = wave_isum(rnp);
    __syncthreads();
    if (lane == 0) {
      for (int q = 0; q < 8; ++q) sw[q] = rs[q];
      sw[8] = rdiv;
      sw[9] = rbm;
      sw[10] = rum;
      sw[11] = rc;
      sw[12] = rrate;
      sl[0] = rca;
      sl[1] = rra;
      sl[2] = nf;
      sl[3] = np;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      RedItem R = {};
      R.carg = R.rarg = 0x7fffffffffffffffLL;
      for (int v = 0; v < NW; ++v) {
        const double* s = sredw + v * 15;
        const long long* l = sredl + v * 4;
        for (int q = 0; q < 8; ++q) R.sum[q] += s[q];
        R.mx[0] = fmax(R.mx[0], s[8]);
        R.mx[1] = fmax(R.mx[1], s[9]);
        R.mx[2] = fmax(R.mx[2], s[10]);
        if (s[11] > R.cmax || (s[11] == R.cmax && l[0] < R.carg)) { R.cmax = s[11]; R.carg = l[0]; }
        if (s[12] > R.rmax || (s[12] == R.rmax && l[1] < R.rarg)) { R.rmax = s[12]; R.rarg = l[1]; }
        R.nonfinite += l[2];
        R.nonpositive += l[3];
      }
      const double dV = b.dx * b.dy * b.dz;   // totals are volume integrals
      for (int q = 0; q < 7; ++q) R.sum[q] *= dV;
      R.darg = 0x7fffffffffffffffLL;   // the diffusion speed: A2, which runs next
      red[item_] = R;
    }
  }
  ZLOOP_END
}

// ---------------------------------------------------------------------------
// S (with T_SMAG): the Smagorinsky rate of eq. nusmag at cell centres,
// [2(S_xx^2 + S_yy^2 + S_zz^2 - (div u)^2/3 + 2(S_xy^2 + S_xz^2 + S_yz^2))]^(1/2),
// added to pass A1's speed-like viscosity as h_min c_smag times it.  The
// off-diagonal strain interpolated from its edge to the centre equals, the
// operators along different axes commuting, S_ab = (D_b ub_a + D_a ub_b) / 2
// with ub_a = aup(u_a) the centred velocities of pass A1 and D_a =
// aup(ddadn(.)): the x and y composites from LDS strips of the front plane
// (queued for the lag of the z ones), the z composites from register
// windows, ddzdn on the z-faces (lag 2), then zup at the centre (lag 5).
// The Smagorinsky term is part of the speed-like viscosity only; the
// constant-viscosity mode has none.
template <class T> static inline bool smag_on(const Phys<T>& ph) {
  return (ph.terms & T_SMAG) && !(ph.nu_const > T(0));
}

template <class T, int TX, int TY, bool PERS>
__global__ __launch_bounds__(TX * TY) void zS(const BoxDev* __restrict__ boxes,
                                              const ZItem* __restrict__ items, int nitems,
                                              const T* __restrict__ ztab, int* __restrict__ queue,
                                              Phys<T> ph, ZWork<T> ws) {
  const T* __restrict__ ubx = ws.q(0);
  const T* __restrict__ uby = ws.q(1);
  const T* __restrict__ ubz = ws.q(2);
  const T* __restrict__ sxx = ws.q(3);
  const T* __restrict__ syy = ws.q(4);
  const T* __restrict__ szz = ws.q(5);
  const T* __restrict__ Dg = ws.arr(WS_D);
  T* __restrict__ nus = ws.arr(WS_NUS);
  using PX5 = Plane<TX, TY, 5, 0>;
  using PY5 = Plane<TX, TY, 0, 5>;
  __shared__ T sUYx[PX5::NP], sUZx[PX5::NP], sUXy[PY5::NP], sUZy[PY5::NP];
  ZLOOP_BEGIN
  PlaneIdx<TX, TY, 5, 0> ix;
  PlaneIdx<TX, TY, 0, 5> iy;
  ix.init(b, it.x0, it.y0);
  iy.init(b, it.x0, it.y0);
  // windows of ub_x, ub_y (slot m = plane r-5+m), of their ddzdn on the
  // z-faces (slot m = face r-7+m), and queues of the x/y composites (slot
  // m = plane r-5+m)
  T wX[6] = {}, wY[6] = {}, wDX[6] = {}, wDY[6] = {};
  T qA[6] = {}, qB[6] = {}, qCX[6] = {}, qCY[6] = {};
  auto comp = [&](const T* s, int step, int base, T hinv) {   // aup(ddadn) over 11 samples
    return op6<0, 1, T>([&](int m) {
      return op6<1, 0, T>([&](int n) { return s[base + (m + n) * step]; }, hinv);
    }, T(0));
  };
  for (int r = it.z0 - 5; r <= it.z1 + 4; ++r) {
    T ux_ = T(0), uy_ = T(0), a = T(0), c = T(0), cx = T(0), cy = T(0);
    if (valid(r)) {
      const int k = kk(r);
      __syncthreads();
      load_plane(sUYx, uby, b, ix, k);
      load_plane(sUZx, ubz, b, ix, k);
      load_plane(sUXy, ubx, b, iy, k);
      load_plane(sUZy, ubz, b, iy, k);
      __syncthreads();
      ux_ = sUXy[PY5::at(tx, ty)];
      uy_ = sUYx[PX5::at(tx, ty)];
      a = comp(sUXy, PY5::W, PY5::at(tx, ty), g.hyi);     // D_y ub_x
      c = comp(sUYx, 1, PX5::at(tx, ty), g.hxi);          // D_x ub_y
      cx = comp(sUZx, 1, PX5::at(tx, ty), g.hxi);         // D_x ub_z
      cy = comp(sUZy, PY5::W, PY5::at(tx, ty), g.hyi);    // D_y ub_z
    }
    push(wX, ux_);
    push(wY, uy_);
    push(qA, a);
    push(qB, c);
    push(qCX, cx);
    push(qCY, cy);
    const int q1 = r - 2;
    T dx_ = T(0), dy_ = T(0);
    if (valid(q1)) {
      dx_ = zwin<1, 0, 6, 3>(wX, q1, wall, N, zj(q1, ZJ_F), zt);
      dy_ = zwin<1, 0, 6, 3>(wY, q1, wall, N, zj(q1, ZJ_F), zt);
    }
    push(wDX, dx_);
    push(wDY, dy_);
    const int q = r - 5;
    if (own && valid(q) && q >= it.z0 && q < it.z1) {
      const long long o = col(q);
      const T sxy = T(0.5) * (qA[0] + qB[0]);
      const T sxz = T(0.5) * (zwin<0, 1, 6, 2>(wDX, q, wall, N, T(0), zt) + qCX[0]);
      const T syz = T(0.5) * (zwin<0, 1, 6, 2>(wDY, q, wall, N, T(0), zt) + qCY[0]);
      const T s11 = sxx[o], s22 = syy[o], s33 = szz[o], D = Dg[o];
      const T s2 = T(2) * (s11 * s11 + s22 * s22 + s33 * s33 - D * D / T(3) +
                           T(2) * (sxy * sxy + sxz * sxz + syz * syz));
      nus[o] += ph.c_smag * zj(q, ZJ_H) * (s2 > T(0) ? sqrt(s2) : T(0));
    }
  }
  ZLOOP_END
}

// ---------------------------------------------------------------------------
// A2: m = max over the MW x MW x MW neighbourhood (MW = 3, or 5 with T_MAX5;
// x, y through LDS, z over a ring of MW x/y-maximum planes), then
// three-cell means along x, y (LDS) and z (register window), floor 1e-30,
// and ln.
//
// RED (the reduction instantiation of mhd_reductions): also the diffusion
// speed max(<nu>, eta_speed h_max / h_min) of eq. courantcond, eta_speed =
// nuB <nu> or eta_const / h_min, and its first maximal cell, into red[item].
template <class T, int TX, int TY, bool PERS, bool RED = false, int MW = 3>
__global__ __launch_bounds__(TX * TY) void zA2(const BoxDev* __restrict__ boxes,
                                               const ZItem* __restrict__ items, int nitems, const T* __restrict__ ztab,
                                               int* __restrict__ queue,
                                               ZWork<T> ws, CPart* __restrict__ cpart,
                                               double nuB = 0.0, double eta_const = 0.0,
                                               RedItem* __restrict__ red = nullptr) {
  static_assert(MW == 3 || MW == 5, "maximum over three or five cells");
  constexpr int MH = MW / 2;
  const T* __restrict__ nus = ws.arr(WS_NUS);
  T* __restrict__ lnt_out = ws.arr(WS_LNT);
  using PN = Plane<TX, TY, MH + 1>;
  using PM = Plane<TX, TY, 1>;
  constexpr int NT = TX * TY;
  __shared__ T sN[PN::NP];
  __shared__ T sMX[MW][PM::NP];
  __shared__ T sM[PM::NP];
  __shared__ double sred[NT];
  ZLOOP_BEGIN
  PlaneIdx<TX, TY, MH + 1> i2;
  i2.init(b, it.x0, it.y0);
  // plane r of nu_s is fetched into registers one iteration ahead (in
  // flight while plane r-1 is worked on); the last fetch repeats the last
  // valid plane
  constexpr int NPF = PlaneIdx<TX, TY, MH + 1>::NPER;
  static_assert(NPF * NT == PN::NP, "plane padding");
  const int rfirst = wall ? max(it.z0 - MH - 1, 0) : it.z0 - MH - 1;
  const int rlast = wall ? min(it.z1 + MH, N - 1) : it.z1 + MH;
  T gN[NPF];
  auto fetch = [&](int r_) {
    const long long pk = b.off + (long long)kk(r_) * pstride;
#pragma unroll
    for (int i = 0; i < NPF; ++i) gN[i] = nus[pk + i2.off[i]];
  };
  fetch(rfirst);
  T wS[3] = {};
  double numax = 0.0;
  double rd = 0.0;
  long long rda = 0x7fffffffffffffffLL;
  for (int r = it.z0 - MH - 1; r <= it.z1 + MH; ++r) {
    if (valid(r)) {
      __syncthreads();
#pragma unroll
      for (int i = 0; i < NPF; ++i) sN[(int)threadIdx.x + i * NT] = gN[i];
      fetch(r < rlast ? r + 1 : r);
      __syncthreads();
      T* dst = sMX[wrapm(r, MW)];
      for (int t = threadIdx.x; t < PM::N; t += NT) {
        const int yy = t / PM::W, xx = t - yy * PM::W;
        const int x = xx - 1, y = yy - 1;
        T m = sN[PN::at(x, y)];
#pragma unroll
        for (int dy = -MH; dy <= MH; ++dy)
#pragma unroll
          for (int dx = -MH; dx <= MH; ++dx) m = fmax(m, sN[PN::at(x + dx, y + dy)]);
        dst[t] = m;
      }
    }
    const int q1 = r - MH;
    T sxy = T(0);
    if (valid(q1)) {
      __syncthreads();
      // maximum over the planes q1 - MH .. q1 + MH that exist
      bool use[MW];
      const T* pl[MW];
#pragma unroll
      for (int d = 0; d < MW; ++d) {
        use[d] = valid(q1 + d - MH);
        pl[d] = sMX[wrapm(q1 + d - MH, MW)];
      }
      for (int t = threadIdx.x; t < PM::N; t += NT) {
        T m = pl[MH][t];
#pragma unroll
        for (int d = 0; d < MW; ++d)
          if (d != MH && use[d]) m = fmax(m, pl[d][t]);
        sM[t] = m;
      }
      __syncthreads();
      T sx[3];
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
        sx[dy + 1] = (sM[PM::at(tx - 1, ty + dy)] + sM[PM::at(tx, ty + dy)] +
                      sM[PM::at(tx + 1, ty + dy)]) / T(3);
      sxy = (sx[0] + sx[1] + sx[2]) / T(3);
    }
    push(wS, sxy);                        // wS slot m = plane r-MH-2+m
    const int q = r - MH - 1;
    if (valid(q) && q >= it.z0 && q < it.z1) {
      T s = wS[1];
      int cnt = 1;
      if (valid(q - 1)) { s = wS[0] + wS[1]; cnt = 2; }
      if (valid(q + 1)) { s = s + wS[2]; ++cnt; }
      T v = s / T(cnt);
      v = v > T(1e-30) ? v : T(1e-30);
      if (own) {
        lnt_out[col(q)] = log(v);
        if (cpart && interior(q)) numax = fmax(numax, (double)v);
        if (RED && interior(q)) {
          const double nu = v;
          const double es = eta_const > 0.0 ? eta_const / b.hmin : nuB * nu;
          const double d = fmax(nu, es * (b.hmax / b.hmin));
          if (d > rd) {
            rd = d;
            rda = b.off + ((long long)q * b.ny + gy) * b.nx + gx;
          }
        }
      }
    }
  }
  if (cpart) {
    const double m = block_max<NT>(numax, sred);
    if (threadIdx.x == 0) cpart[item_].numax = m;
  }
  if constexpr (RED) {
    wave_maxarg(rd, rda);
    __syncthreads();
    if (threadIdx.x % 64 == 0) {
      sred[threadIdx.x / 64] = rd;
      reinterpret_cast<long long*>(sred)[NT / 64 + threadIdx.x / 64] = rda;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double d = 0.0;
      long long a = 0x7fffffffffffffffLL;
      for (int v = 0; v < NT / 64; ++v) {
        const double dv = sred[v];
        const long long av = reinterpret_cast<long long*>(sred)[NT / 64 + v];
        if (dv > d || (dv == d && av < a)) { d = dv; a = av; }
      }
      red[item_].dmax = d;
      red[item_].darg = a;
    }
  }
  ZLOOP_END
}

// ---------------------------------------------------------------------------
// Q: x-directed and y-directed edges (at z = k-1/2), the z-face energy flux
// Hz and the centre terms Gzz = tau_zz - zup(p_z) zup(u_z) - P and
// Czz = tau_zz S_zz.  Outputs (QOUT_*):
//   y-edge (i-1/2, j, k-1/2): Gxz, Gzx, Ey, Lxy, Lzy, Qy
//   x-edge (i, j-1/2, k-1/2): Gyz, Gzy, Ex, Lyx, Lzx, Qx
//   Hz (z-face), Gzz, Czz (centre)
// QM selects the output groups of a launch: QM_EDGES (both edges, which need
// x/y stencils through LDS) and QM_ZC (z-face and centre, pointwise in x/y).
// The stage runs one launch of each: apart, each needs far fewer registers
// (float64: occupancy 1 -> 2 and 3), for four arrays read twice.
constexpr unsigned QM_EDGES = 1u, QM_ZC = 2u;
// with QM_ZC: dP/dz through ln(P / P_aver) (eq. pressure)
constexpr unsigned QM_LNP = 4u;
// quenching: only the raw stress components of the selected groups
// (tau_xz, tau_yz; tau_zz), into the workspace arrays q(TAU_*)
constexpr unsigned QM_TAU = 8u;
template <class T, int TX, int TY, bool PERS, unsigned QM>
__global__ __launch_bounds__(TX * TY) void zQ(const BoxDev* __restrict__ boxes,
                                              const ZItem* __restrict__ items, int nitems, const T* __restrict__ ztab,
                                               int* __restrict__ queue,
                                              CP8<T> f, Phys<T> ph, ZWork<T> ws,
                                              const T* __restrict__ lnavg,
                                              const T* __restrict__ lnpav) {
  const T* __restrict__ uzg = ws.arr(WS_UZ);
  const T* __restrict__ lntg = ws.arr(WS_LNT);
  const T* __restrict__ Dg = ws.arr(WS_D);
  using P3 = Plane<TX, TY, 3>;
  constexpr bool kE = QM & QM_EDGES, kZ = QM & QM_ZC, kT = QM & QM_TAU;
  constexpr int NPL = kE ? P3::NP : 1;
  constexpr int NPB = kE && !kT ? P3::NP : 1;
  __shared__ T sR[NPL], sL[NPL];
  __shared__ T sUZ[3][NPL], sBZ[3][NPB], sPZ[3][NPB];
  const T* __restrict__ tq = ws.tq;
  ZLOOP_BEGIN
  PlaneIdx<TX, TY, 3> i3;
  i3.init(b, it.x0, it.y0);
  const unsigned tm = ph.terms;
  const bool visc = tm & T_VISC, res = tm & T_RESIST, ind = tm & T_INDUCT, lor = tm & T_LORENTZ,
             adv = tm & T_ADV, pres = tm & T_PRES, ediff = tm & T_EDIFF;
  const bool ediffav = ediff && (tm & T_EDIFFAV);
  const bool need_nu = visc || (res && !(ph.eta_const > T(0)));
  // windows: slot m = plane r-5+m
  T wRX[6] = {}, wLX[6] = {}, wPX[6] = {}, wUX[6] = {}, wBX[6] = {};
  T wRY[6] = {}, wLY[6] = {}, wPY[6] = {}, wUY[6] = {}, wBY[6] = {};
  T wPZ[6] = {}, wUZ[6] = {}, wE[6] = {}, wRho[6] = {}, wNu[6] = {}, wEm[6] = {}, wLem[6] = {};
  // eq. pressure (QM_LNP): ln(P / P_aver) and ln P_aver
  constexpr bool kL = QM & QM_LNP;
  T wLq[6] = {}, wLpa[6] = {};
  const T inv_mu = ph.inv_mu;
  // The ring planes (u_z; B_z and p_z) of plane r are fetched into
  // registers one iteration ahead, after plane r-1's own-column loads, so
  // that they are in flight while plane r-1 is worked on.  Planes past the
  // last valid one are not fetched: the last fetch repeats that plane.
  constexpr int N3 = PlaneIdx<TX, TY, 3>::NPER;
  static_assert(N3 * TX * TY == P3::NP, "plane padding");
  const int rfirst = wall ? max(it.z0 - 3, 0) : it.z0 - 3;
  const int rlast = wall ? min(it.z1 + 2, N - 1) : it.z1 + 2;
  T gU[N3], gB[N3], gP[N3];
  auto fetch = [&](int r_) {
    const long long pk = b.off + (long long)kk(r_) * pstride;
#pragma unroll
    for (int i = 0; i < N3; ++i) {
      gU[i] = uzg[pk + i3.off[i]];
      if constexpr (!kT) {
        gB[i] = f.p[7][pk + i3.off[i]];
        gP[i] = f.p[3][pk + i3.off[i]];
      }
    }
  };
  if constexpr (kE) fetch(rfirst);
  // The z-face and centre launch likewise fetches plane r's own-column
  // values one iteration ahead, and in every iteration div u of the next
  // iteration's centre plane (at a valid plane whether or not that one is:
  // unused then).
  T zP_ = T(0), zU_ = T(0), zR_ = T(0), zL_ = T(0), zE_ = T(0), zD_ = T(0);
  auto fetchz = [&](int r_) {
    const long long o_ = col(r_);
    zP_ = f.p[3][o_];
    zU_ = uzg[o_];
    zR_ = f.p[0][o_];
    zL_ = lntg[o_];
    zE_ = f.p[4][o_];
  };
  if constexpr (kZ && !kE) fetchz(rfirst);
  for (int r = it.z0 - 3; r <= it.z1 + 2; ++r) {
    const T dq2 = zD_;   // div u at plane r - 3 (the centre plane below)
    T rx = T(0), lx = T(0), px = T(0), ux = T(0), bxv = T(0);
    T ry = T(0), ly = T(0), py = T(0), uy = T(0), byv = T(0);
    T pzv = T(0), uzv = T(0), ev = T(0), rhov = T(0), nuv = T(0), em = T(0), lem = T(0);
    T lq = T(0), lpa = T(0);
    if (valid(r)) {
      const int k = kk(r), sl = wrapm(r, 3);
      const long long o = col(r);
      if constexpr (kE) {
        __syncthreads();
        load_plane(sR, f.p[0], b, i3, k);
        load_plane(sL, lntg, b, i3, k);
#pragma unroll
        for (int i = 0; i < N3; ++i) {
          sUZ[sl][(int)threadIdx.x + i * TX * TY] = gU[i];
          if constexpr (!kT) {
            sBZ[sl][(int)threadIdx.x + i * TX * TY] = gB[i];
            sPZ[sl][(int)threadIdx.x + i * TX * TY] = gP[i];
          }
        }
        px = f.p[1][o];
        py = f.p[2][o];
        if constexpr (!kT) {
          bxv = f.p[5][o];
          byv = f.p[6][o];
        }
        fetch(r < rlast ? r + 1 : r);
        __syncthreads();
        rx = op6<0, 0, T>([&](int m) { return sR[P3::at(tx + m, ty)]; }, T(0));
        ry = op6<0, 0, T>([&](int m) { return sR[P3::at(tx, ty + m)]; }, T(0));
        lx = op6<0, 0, T>([&](int m) { return sL[P3::at(tx + m, ty)]; }, T(0));
        ly = op6<0, 0, T>([&](int m) { return sL[P3::at(tx, ty + m)]; }, T(0));
        ux = px / rx;
        uy = py / ry;
      }
      if constexpr (kZ) {
        // own column only: from LDS when the planes are there
        if constexpr (kE && !kT) {
          pzv = sPZ[sl][P3::at(tx, ty)];
          uzv = sUZ[sl][P3::at(tx, ty)];
          rhov = sR[P3::at(tx, ty)];
          nuv = exp(sL[P3::at(tx, ty)]);
          ev = f.p[4][o];
        } else {
          pzv = zP_;
          uzv = zU_;
          rhov = zR_;
          nuv = exp(zL_);
          ev = zE_;
          fetchz(r < rlast ? r + 1 : r);
        }
        em = ev / rhov;
        lem = log(em);
        // eq. ediffav: the z flux differentiates ln e_m - ln <e_m>
        if (ediffav) lem -= lnavg[b.poff + k];
        if constexpr (kL) {
          lpa = lnpav[b.poff + k];
          lq = log(ph.gamma1 * ev) - lpa;
        }
      }
    }
    if constexpr (kZ && !kE) zD_ = Dg[col(valid(r - 2) ? r - 2 : rfirst)];
    push(wRX, rx); push(wLX, lx); push(wPX, px); push(wUX, ux); push(wBX, bxv);
    push(wRY, ry); push(wLY, ly); push(wPY, py); push(wUY, uy); push(wBY, byv);
    push(wPZ, pzv); push(wUZ, uzv); push(wE, ev); push(wRho, rhov); push(wNu, nuv);
    push(wEm, em); push(wLem, lem);
    if constexpr (kL) {
      push(wLq, lq);
      push(wLpa, lpa);
    }

    // edges and z-face of plane q = r - 2 (window slot 3)
    const int q = r - 2;
    if (valid(q) && q >= it.z0 && q < it.z1) {
      const int sq = wrapm(q, 3);
      const T* UZ = sUZ[sq];
      const T* BZ = sBZ[sq];
      const T* PZ = sPZ[sq];
      const long long o = col(q);
      // second-order switch: the strain of the x- and y-edges (the end face
      // of a wall axis copies its neighbour's z derivative)
      const unsigned fl = (kE && ws.rgh) ? (unsigned)ws.rgh[o] : 0u;
      auto dz2 = [&](const T (&w)[6]) {
        return (wall && q == 0) ? (w[4] - w[3]) * zj(q, ZJ_F) : (w[3] - w[2]) * zj(q, ZJ_F);
      };
      auto s_xz = [&](T dzUX, T dxUZ) {
        if (fl & RG_YE) return T(0.5) * (dz2(wUX) + (UZ[P3::at(tx, ty)] - UZ[P3::at(tx - 1, ty)]) * g.hxi);
        return T(0.5) * (dzUX + dxUZ);
      };
      auto s_yz = [&](T dzUY, T dyUZ) {
        if (fl & RG_XE) return T(0.5) * (dz2(wUY) + (UZ[P3::at(tx, ty)] - UZ[P3::at(tx, ty - 1)]) * g.hyi);
        return T(0.5) * (dzUY + dyUZ);
      };
      // ---- raw stress only (quenching)
      if constexpr (kE && kT) {
        const T dxUZ = op6<1, 0, T>([&](int m) { return UZ[P3::at(tx + m, ty)]; }, g.hxi);
        const T dyUZ = op6<1, 0, T>([&](int m) { return UZ[P3::at(tx, ty + m)]; }, g.hyi);
        const T sxz = s_xz(zwin<1, 0, 6, 3>(wUX, q, wall, N, zj(q, ZJ_F), zt), dxUZ);
        const T syz = s_yz(zwin<1, 0, 6, 3>(wUY, q, wall, N, zj(q, ZJ_F), zt), dyUZ);
        if (own) {
          ws.q(TAU_XZ)[o] = zwin<0, 0, 6, 3>(wRX, q, wall, N, T(0), zt) *
                            (zj(q, ZJ_LXZ) * exp(zwin<0, 0, 6, 3>(wLX, q, wall, N, T(0), zt))) * sxz;
          ws.q(TAU_YZ)[o] = zwin<0, 0, 6, 3>(wRY, q, wall, N, T(0), zt) *
                            (zj(q, ZJ_LYZ) * exp(zwin<0, 0, 6, 3>(wLY, q, wall, N, T(0), zt))) * syz;
        }
      }
      // ---- y-edge
      if constexpr (kE && !kT) {
        const T zRX = zwin<0, 0, 6, 3>(wRX, q, wall, N, T(0), zt);
        const T zPX = zwin<0, 0, 6, 3>(wPX, q, wall, N, T(0), zt);
        const T zUX = zwin<0, 0, 6, 3>(wUX, q, wall, N, T(0), zt);
        const T dzUX = zwin<1, 0, 6, 3>(wUX, q, wall, N, zj(q, ZJ_F), zt);
        const T zBX = zwin<0, 0, 6, 3>(wBX, q, wall, N, T(0), zt);
        const T dzBX = zwin<1, 0, 6, 3>(wBX, q, wall, N, zj(q, ZJ_F), zt);
        const T xUZ = op6<0, 0, T>([&](int m) { return UZ[P3::at(tx + m, ty)]; }, T(0));
        const T dxUZ = op6<1, 0, T>([&](int m) { return UZ[P3::at(tx + m, ty)]; }, g.hxi);
        const T xBZ = op6<0, 0, T>([&](int m) { return BZ[P3::at(tx + m, ty)]; }, T(0));
        const T dxBZ = op6<1, 0, T>([&](int m) { return BZ[P3::at(tx + m, ty)]; }, g.hxi);
        const T xPZ = op6<0, 0, T>([&](int m) { return PZ[P3::at(tx + m, ty)]; }, T(0));
        T nxz = T(0), txz = T(0), sxz = T(0);
        if (need_nu) nxz = zj(q, ZJ_LXZ) * exp(zwin<0, 0, 6, 3>(wLX, q, wall, N, T(0), zt));
        if (visc) {
          sxz = s_xz(dzUX, dxUZ);
          txz = tq ? tq[TAU_XZ * ws.stride + o] : zRX * nxz * sxz;
        }
        const T jy = dzBX - dxBZ;
        const T eta = ph.eta_const > T(0) ? ph.eta_const : ph.nuB * nxz;
        T ey = T(0);
        if (ind) ey = ey - (xUZ * zBX - zUX * xBZ);
        if (res) ey = ey + eta * jy;
        T gxz = txz, gzx = txz;
        if (adv) {
          gxz = gxz - zPX * xUZ;
          gzx = gzx - xPZ * zUX;
        }
        T qy = visc ? T(2) * txz * sxz : T(0);
        if (res) qy = qy + eta * jy * jy * inv_mu;
        if (own) {
          ws.q(QOUT_GXZ)[o] = gxz;
          ws.q(QOUT_GZX)[o] = gzx;
          ws.q(QOUT_EY)[o] = ey;
          ws.q(QOUT_LXY)[o] = lor ? jy * xBZ : T(0);
          ws.q(QOUT_LZY)[o] = lor ? jy * zBX : T(0);
          ws.q(QOUT_QY)[o] = qy;
        }
      }
      // ---- x-edge
      if constexpr (kE && !kT) {
        const T zRY = zwin<0, 0, 6, 3>(wRY, q, wall, N, T(0), zt);
        const T zPY = zwin<0, 0, 6, 3>(wPY, q, wall, N, T(0), zt);
        const T zUY = zwin<0, 0, 6, 3>(wUY, q, wall, N, T(0), zt);
        const T dzUY = zwin<1, 0, 6, 3>(wUY, q, wall, N, zj(q, ZJ_F), zt);
        const T zBY = zwin<0, 0, 6, 3>(wBY, q, wall, N, T(0), zt);
        const T dzBY = zwin<1, 0, 6, 3>(wBY, q, wall, N, zj(q, ZJ_F), zt);
        const T yUZ = op6<0, 0, T>([&](int m) { return UZ[P3::at(tx, ty + m)]; }, T(0));
        const T dyUZ = op6<1, 0, T>([&](int m) { return UZ[P3::at(tx, ty + m)]; }, g.hyi);
        const T yBZ = op6<0, 0, T>([&](int m) { return BZ[P3::at(tx, ty + m)]; }, T(0));
        const T dyBZ = op6<1, 0, T>([&](int m) { return BZ[P3::at(tx, ty + m)]; }, g.hyi);
        const T yPZ = op6<0, 0, T>([&](int m) { return PZ[P3::at(tx, ty + m)]; }, T(0));
        T nyz = T(0), tyz = T(0), syz = T(0);
        if (need_nu) nyz = zj(q, ZJ_LYZ) * exp(zwin<0, 0, 6, 3>(wLY, q, wall, N, T(0), zt));
        if (visc) {
          syz = s_yz(dzUY, dyUZ);
          tyz = tq ? tq[TAU_YZ * ws.stride + o] : zRY * nyz * syz;
        }
        const T jx = dyBZ - dzBY;
        const T eta = ph.eta_const > T(0) ? ph.eta_const : ph.nuB * nyz;
        T ex = T(0);
        if (ind) ex = ex - (zUY * yBZ - yUZ * zBY);
        if (res) ex = ex + eta * jx;
        T gyz = tyz, gzy = tyz;
        if (adv) {
          gyz = gyz - zPY * yUZ;
          gzy = gzy - yPZ * zUY;
        }
        T qx = visc ? T(2) * tyz * syz : T(0);
        if (res) qx = qx + eta * jx * jx * inv_mu;
        if (own) {
          ws.q(QOUT_GYZ)[o] = gyz;
          ws.q(QOUT_GZY)[o] = gzy;
          ws.q(QOUT_EX)[o] = ex;
          ws.q(QOUT_LYX)[o] = lor ? jx * yBZ : T(0);
          ws.q(QOUT_LZX)[o] = lor ? jx * zBY : T(0);
          ws.q(QOUT_QX)[o] = qx;
        }
      }
      // ---- z-face energy flux: -zdn(e) u_z + nuE zdn(rho) dz zdn(nu) zdn(e_m) ddzdn(ln e_m)
      if constexpr (kZ && !kT) {
        T hz = T(0);
        if (adv) hz = -zwin<0, 0, 6, 3>(wE, q, wall, N, T(0), zt) * wUZ[3];
        if (ediff)
          hz = hz + ph.nuE * zwin<0, 0, 6, 3>(wRho, q, wall, N, T(0), zt) *
                        (zj(q, ZJ_LZF) * zwin<0, 0, 6, 3>(wNu, q, wall, N, T(0), zt)) *
                        zwin<0, 0, 6, 3>(wEm, q, wall, N, T(0), zt) *
                        zwin<1, 0, 6, 3>(wLem, q, wall, N, zj(q, ZJ_F), zt);
        if (own) {
          ws.q(QOUT_HZ)[o] = hz;
          // pressure gradient on its own: folded into the flux, a pressure
          // of order one would swamp the much smaller stresses in float32
          T dpz = T(0);
          if (pres) {
            if constexpr (kL)
              dpz = exp(zwin<0, 0, 6, 3>(wLpa, q, wall, N, T(0), zt)) *
                    exp(zwin<0, 0, 6, 3>(wLq, q, wall, N, T(0), zt)) *
                    (zwin<1, 0, 6, 3>(wLq, q, wall, N, zj(q, ZJ_F), zt) +
                     zwin<1, 0, 6, 3>(wLpa, q, wall, N, zj(q, ZJ_F), zt));
            else
              dpz = ph.gamma1 * zwin<1, 0, 6, 3>(wE, q, wall, N, zj(q, ZJ_F), zt);
          }
          ws.q(QOUT_DPZ)[o] = dpz;
        }
      }
    }
    // centre terms of plane q2 = r - 3 (window slot 2)
    const int q2 = r - 3;
    if (kZ && valid(q2) && q2 >= it.z0 && q2 < it.z1) {
      const long long o = col(q2);
      // second-order switch at the centre: S_zz and the stress's div u
      const bool o2 = ws.rgh && ((unsigned)ws.rgh[o] & RG_C);
      const T jq2 = zj(q2, ZJ_C);
      const T szz = !o2 ? zwin<1, 1, 6, 2>(wUZ, q2, wall, N, jq2, zt)
                        : ((wall && q2 == N - 1) ? (wUZ[2] - wUZ[1]) * jq2 : (wUZ[3] - wUZ[2]) * jq2);
      const T Dt = o2 ? ws.arr(WS_D2)[o] : (kE ? Dg[o] : dq2);
      if constexpr (kT) {
        if (own) ws.q(TAU_ZZ)[o] = wRho[2] * (zj(q2, ZJ_LZZ) * wNu[2]) * (szz + ph.c1 * Dt);
        continue;
      }
      T gzz = T(0), czz = T(0);
      if (visc) {
        const T tzz = tq ? tq[TAU_ZZ * ws.stride + o] : wRho[2] * (zj(q2, ZJ_LZZ) * wNu[2]) * (szz + ph.c1 * Dt);
        gzz = tzz;
        czz = tzz * szz;
      }
      if (adv) gzz = gzz - zwin<0, 1, 6, 2>(wPZ, q2, wall, N, T(0), zt) * zwin<0, 1, 6, 2>(wUZ, q2, wall, N, T(0), zt);
      if (own) {
        ws.q(QOUT_GZZ)[o] = gzz;
        ws.q(QOUT_CZZ)[o] = czz;
      }
    }
  }
  ZLOOP_END
}

// ---------------------------------------------------------------------------
// P: everything that needs only x/y stencils, once per cell at its own
// column: the z-directed edge (x-1/2, y-1/2) quantities Gxy, Gyx, Ez, Lxz,
// Lyz, Qz (as in Q), the centre terms Gxx = tau_xx - xup(p_x) xup(u_x),
// Gyy, Qc = tau_xx S_xx + tau_yy S_yy - P div u, the x/y-face energy
// fluxes Hx, Hy (eq. ien, eq. ediffuse) and the x/y-face pressure
// gradients, kept out of the fluxes (face_dp).
// TAU (quenching): only the raw stress components tau_xy, tau_xx, tau_yy,
// into the workspace arrays q(TAU_*).
template <class T, int TX, int TY, bool PERS, bool TAU = false>
__global__ __launch_bounds__(TX * TY) void zP(const BoxDev* __restrict__ boxes,
                                              const ZItem* __restrict__ items, int nitems, const T* __restrict__ ztab,
                                               int* __restrict__ queue,
                                              CP8<T> f, Phys<T> ph, ZWork<T> ws) {
  const T* __restrict__ lntg = ws.arr(WS_LNT);
  const T* __restrict__ Dg = ws.arr(WS_D);
  const T* __restrict__ uzg = ws.arr(WS_UZ);
  const T* __restrict__ lnpav = ws.lnpav;
  using P6 = Plane<TX, TY, 6>;
  using P3 = Plane<TX, TY, 3>;
  constexpr int NT = TX * TY;
  // halo-3 planes: 0 px 1 py 2 e 3 Bx 4 By 5 ln nu | derived: 6 ux 7 uy 8 nu
  // 9 e_m 10 ln e_m 11 xdn(rho) 12 ydn(rho) 13 xdn(ln nu)
  constexpr int NS = 14;
  __shared__ T sR[P6::NP];
  __shared__ T s3[NS * P3::NP];
  ZLOOP_BEGIN
  PlaneIdx<TX, TY, 6> i6;
  PlaneIdx<TX, TY, 3> i3;
  i6.init(b, it.x0, it.y0);
  i3.init(b, it.x0, it.y0);
  const unsigned tm = ph.terms;
  auto S = [&](int q, int x, int y) -> T& { return s3[q * P3::NP + P3::at(x, y)]; };
  // Some planes of z plane k are fetched into registers one iteration
  // ahead, so that their loads are in flight while plane k-1 is worked on:
  // B_x, B_y and ln <nu> (the stress alone, TAU, reads neither e nor the
  // magnetic field: there p_x, p_y and ln <nu>).  The others are loaded in
  // the iteration: fetching them too would cost the float32 64x8 launch a
  // wave per SIMD.
  constexpr int N3 = PlaneIdx<TX, TY, 3>::NPER;
  static_assert(N3 * NT == P3::NP, "plane padding");
  auto has3 = [](int q) { return !TAU || q < 2 || q == 5; };
  auto ahead = [](int q) { return TAU ? (q < 2 || q == 5) : q >= 3; };
  const T* __restrict__ src3[6] = {f.p[1], f.p[2], f.p[4], f.p[5], f.p[6], lntg};
  T g3[6][N3];
  auto fetch = [&](int k) {
    const long long pk = b.off + (long long)k * pstride;
#pragma unroll
    for (int q = 0; q < 6; ++q)
      if (ahead(q)) {
#pragma unroll
        for (int i = 0; i < N3; ++i) g3[q][i] = src3[q][pk + i3.off[i]];
      }
  };
  fetch(it.z0);
  for (int k = it.z0; k < it.z1; ++k) {
    __syncthreads();
    load_plane(sR, f.p[0], b, i6, k);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      if (ahead(q)) {
#pragma unroll
        for (int i = 0; i < N3; ++i) s3[q * P3::NP + (int)threadIdx.x + i * NT] = g3[q][i];
      } else if (has3(q)) {
        load_plane(&S(q, -3, -3), src3[q], b, i3, k);
      }
    }
    // this column's div u (an in-box address for every thread), then plane
    // k + 1 (the last plane fetches itself again: no branch around loads)
    const T Dc = Dg[colo + (long long)k * pstride];
    fetch(k + 1 < it.z1 ? k + 1 : k);
    __syncthreads();
    for (int t = threadIdx.x; t < P3::N; t += NT) {
      const int yy = t / P3::W, xx = t - yy * P3::W;
      const int x = xx - 3, y = yy - 3;
      const T rxd = op6<0, 0, T>([&](int m) { return sR[P6::at(x + m, y)]; }, T(0));
      const T ryd = op6<0, 0, T>([&](int m) { return sR[P6::at(x, y + m)]; }, T(0));
      const T rc = sR[P6::at(x, y)];
      s3[6 * P3::NP + t] = s3[0 * P3::NP + t] / rxd;
      s3[7 * P3::NP + t] = s3[1 * P3::NP + t] / ryd;
      s3[8 * P3::NP + t] = exp(s3[5 * P3::NP + t]);
      if constexpr (!TAU) {
        const T emv = s3[2 * P3::NP + t] / rc;
        s3[9 * P3::NP + t] = emv;
        s3[10 * P3::NP + t] = log(emv);
      }
      s3[11 * P3::NP + t] = rxd;
      s3[12 * P3::NP + t] = ryd;
      // xdn(ln nu) is only needed on the own columns' y-strip
      if (x >= 0 && x < TX)
        s3[13 * P3::NP + t] = op6<0, 0, T>([&](int m) { return s3[5 * P3::NP + t + m]; }, T(0));
    }
    __syncthreads();
    if (!own) continue;
    const int x = tx, y = ty;
    const long long o = colo + (long long)k * pstride;
    const T lpa = (tm & T_LNP) ? lnpav[b.poff + k] : T(0);
    // derived planes by id (mhd_zstage.hpp); ln(P / P_aver) on the fly
    auto SA = [&](int q, int xx, int yy) -> T {
      if (q == DQ_RHO) return sR[P6::at(xx, yy)];
      if (q == DQ_D) return Dc;    // read at the own point only
      if (q == DQ_LQ) return log(ph.gamma1 * S(DQ_E, xx, yy)) - lpa;
      return S(q, xx, yy);
    };
    // second-order switch: this cell's flags and its second-order div u
    // (also for pass Q's tau_zz; the end plane of a wall axis copies its
    // neighbour's z derivative)
    unsigned fl = 0;
    T D2 = T(0);
    if (ws.rgh) {
      fl = (unsigned)ws.rgh[o];
      const int kp = (wall && k == N - 1) ? k - 1 : k;
      D2 = (S(DQ_UX, x + 1, y) - S(DQ_UX, x, y)) * g.hxi + (S(DQ_UY, x, y + 1) - S(DQ_UY, x, y)) * g.hyi +
           (uzg[col(kp + 1)] - uzg[col(kp)]) * zj(k, ZJ_C);
      ws.arr(WS_D2)[o] = D2;
    }
    if constexpr (TAU) {
      T sxx, syy, txx, tyy;
      centre_tau<T>(SA, x, y, g, ph, sxx, syy, txx, tyy, fl & RG_C, D2);
      ws.q(TAU_XY)[o] = zedge_tau<T>(SA, x, y, g, fl & RG_ZE);
      ws.q(TAU_XX)[o] = txx;
      ws.q(TAU_YY)[o] = tyy;
      continue;
    }
    T gxy, gyx, ez, lxz, lyz, qz, gxx, gyy, qc, dpx, dpy;
    const T* tq = ws.tq;
    zedge_q<T>(SA, x, y, g, ph, gxy, gyx, ez, lxz, lyz, qz, tq ? tq + TAU_XY * ws.stride + o : nullptr,
               fl & RG_ZE);
    centre_q<T>(SA, x, y, g, ph, gxx, gyy, qc, tq ? tq + TAU_XX * ws.stride + o : nullptr, ws.stride,
                fl & RG_C, D2);
    face_dp<T>(SA, x, y, g, ph, (tm & T_LNP) ? T(exp(lpa)) : T(0), dpx, dpy);
    ws.pq(POUT_GXY)[o] = gxy;
    ws.pq(POUT_GYX)[o] = gyx;
    ws.pq(POUT_EZ)[o] = ez;
    ws.pq(POUT_LXZ)[o] = lxz;
    ws.pq(POUT_LYZ)[o] = lyz;
    ws.pq(POUT_QZ)[o] = qz;
    ws.pq(POUT_GXX)[o] = gxx;
    ws.pq(POUT_GYY)[o] = gyy;
    ws.pq(POUT_QC)[o] = qc;
    ws.pq(POUT_DPX)[o] = dpx;
    ws.pq(POUT_DPY)[o] = dpy;
    ws.pq(POUT_HX)[o] = xface_h<T>(SA, x, y, g, ph);
    ws.pq(POUT_HY)[o] = yface_h<T>(SA, x, y, g, ph);
  }
  ZLOOP_END
}

// ---------------------------------------------------------------------------
// Second-order switch (Section 3 after eq. itv): the flags (RG_*) of every
// cell into workspace array WS_RGH.  A cell is rough where some axis's
// absolute second difference of ln rho or ln e_m exceeds d2_lim (none across
// the ends of a wall-bounded axis).  ln rho and ln e_m of planes r-2, r-1, r
// sit in an LDS ring (halo 2); the roughness of plane r-1 on the tile and a
// one-cell rim goes to an LDS ring of two planes (an absent plane is
// smooth); the flags of plane r-1 collect the cells touching each position.
template <class T, int TX, int TY, bool PERS>
__global__ __launch_bounds__(TX * TY) void zRough(const BoxDev* __restrict__ boxes,
                                                  const ZItem* __restrict__ items, int nitems,
                                                  const T* __restrict__ ztab, int* __restrict__ queue,
                                                  CP8<T> f, Phys<T> ph, ZWork<T> ws) {
  using P2 = Plane<TX, TY, 2>;
  using P1 = Plane<TX, TY, 1>;
  using I2 = PlaneIdx<TX, TY, 2>;
  constexpr int NT = TX * TY;
  __shared__ T sLR[3][P2::NP], sLE[3][P2::NP];
  __shared__ unsigned char sG[2][P1::NP];
  T* __restrict__ out = ws.arr(WS_RGH);
  ZLOOP_BEGIN
  I2 i2;
  i2.init(b, it.x0, it.y0);
  // rho and e of plane r are fetched into registers one iteration ahead
  // (clamped to the valid planes: the loads need no branch)
  const int r0 = it.z0 - 2;
  const int rlo = wall ? max(r0, 0) : r0;
  const int rhi = wall ? min(it.z1, N - 1) : it.z1;
  auto clampr = [&](int r_) { return r_ < rlo ? rlo : (r_ > rhi ? rhi : r_); };
  T gr[I2::NPER], ge[I2::NPER];
  auto fetch = [&](int r_) {
    const long long pk = b.off + (long long)kk(r_) * pstride;
#pragma unroll
    for (int i = 0; i < I2::NPER; ++i) {
      gr[i] = f.p[0][pk + i2.off[i]];
      ge[i] = f.p[4][pk + i2.off[i]];
    }
  };
  fetch(clampr(r0));
  for (int r = it.z0 - 2; r <= it.z1; ++r) {
    __syncthreads();
    if (valid(r)) {
      const int sl = wrapm(r, 3);
#pragma unroll
      for (int i = 0; i < I2::NPER; ++i) {
        const int t = (int)threadIdx.x + i * NT;
        sLR[sl][t] = log(gr[i]);
        sLE[sl][t] = log(ge[i] / gr[i]);
      }
    }
    fetch(clampr(r + 1));
    __syncthreads();
    const int p = r - 1;
    if (r < it.z0) continue;
    unsigned char* G = sG[wrapm(p, 2)];
    if (valid(p)) {
      const int s0 = wrapm(p, 3), sm = wrapm(p - 1, 3), sp = wrapm(p + 1, 3);
      const bool zok = valid(p - 1) && valid(p + 1);
      for (int t = threadIdx.x; t < P1::N; t += NT) {
        const int yy = t / P1::W, xx = t - yy * P1::W;
        const int x = xx - 1, y = yy - 1;
        T m = T(0);
        for (int v = 0; v < 2; ++v) {
          const T* A = v ? sLE[s0] : sLR[s0];
          const T c = A[P2::at(x, y)];
          m = fmax(m, fabs(A[P2::at(x + 1, y)] - T(2) * c + A[P2::at(x - 1, y)]));
          m = fmax(m, fabs(A[P2::at(x, y + 1)] - T(2) * c + A[P2::at(x, y - 1)]));
          if (zok) {
            const T* Am = v ? sLE[sm] : sLR[sm];
            const T* Ap = v ? sLE[sp] : sLR[sp];
            m = fmax(m, fabs(Ap[P2::at(x, y)] - T(2) * c + Am[P2::at(x, y)]));
          }
        }
        G[t] = m > ph.d2_lim ? 1 : 0;
      }
    } else {
      for (int t = threadIdx.x; t < P1::NP; t += NT) G[t] = 0;
    }
    __syncthreads();
    if (own && p >= it.z0 && p < it.z1 && valid(p)) {
      const unsigned char* G1 = sG[wrapm(p - 1, 2)];
      auto g0 = [&](int dx, int dy) { return G[P1::at(tx + dx, ty + dy)] != 0; };
      auto g1 = [&](int dx, int dy) { return G1[P1::at(tx + dx, ty + dy)] != 0; };
      unsigned fl = 0;
      if (g0(0, 0)) fl |= RG_C;
      if (g0(0, 0) || g0(0, -1) || g1(0, 0) || g1(0, -1)) fl |= RG_XE;
      if (g0(0, 0) || g0(-1, 0) || g1(0, 0) || g1(-1, 0)) fl |= RG_YE;
      if (g0(0, 0) || g0(-1, 0) || g0(0, -1) || g0(-1, -1)) fl |= RG_ZE;
      out[col(p)] = T(fl);
    }
  }
  ZLOOP_END
}

// ---------------------------------------------------------------------------
// Quenching of the viscous stress (Section 6.2, eq. quench): component
// blockIdx.y of the raw stress (workspace array q(c)) into the quenched one
// (array WS_TQ0 + c): tau min(max of q over the 3x3x3 neighbourhood, q_lim),
// q = D2 / (|tau| + D2 / q_max), D2 the sum over the axes of the absolute
// second differences (none across the ends of a wall-bounded z axis), q = 0
// where tau and D2 vanish.  The raw planes sit in an LDS ring of four
// (halo 2); each plane is fetched into registers two iterations ahead, so
// its loads are in flight while the two planes before it are worked on.  q of
// plane r-1 on the tile and a one-cell rim goes to LDS, its in-plane
// maximum over 3x3 cells into a z window (q >= 0, so a plane that does not
// exist counts as 0), and plane r-2 is finished.
template <class T, int TX, int TY>
__global__ __launch_bounds__(TX * TY) void zQn(const BoxDev* __restrict__ boxes,
                                               const ZItem* __restrict__ items, int nitems,
                                               const T* __restrict__ ztab, Phys<T> ph, ZWork<T> ws) {
  constexpr bool PERS = false;
  int* queue = nullptr;
  using P2 = Plane<TX, TY, 2>;
  using P1 = Plane<TX, TY, 1>;
  using I2 = PlaneIdx<TX, TY, 2>;
  static_assert(I2::NPER * I2::NT == P2::NP, "plane padding");
  constexpr int NT = TX * TY;
  // ring slot of plane r: wrapm(r, 4).  Plane r overwrites plane r-4, last
  // read two iterations earlier, with two barriers in between; so the
  // writes need no barrier of their own.
  __shared__ T sT[4][P2::NP];
  __shared__ T sQ[P1::NP];
  const int c = (int)blockIdx.y;
  const T* __restrict__ tin = ws.q(c);
  T* __restrict__ tout = ws.arr(WS_TQ0 + c);
  ZLOOP_BEGIN
  I2 i2;
  i2.init(b, it.x0, it.y0);
  // two register sets, each holding a plane fetched two iterations ahead
  T preA[I2::NPER], preB[I2::NPER];
  auto fetch = [&](T (&d)[I2::NPER], int r) {
    const T* __restrict__ s = tin + b.off + (long long)kk(r) * pstride;
#pragma unroll
    for (int i = 0; i < I2::NPER; ++i) d[i] = s[i2.off[i]];
  };
  // planes outside a wall-bounded axis are not fetched: the fetches are
  // clamped to the valid planes (unconditional, so that the compiler can
  // count the loads in flight and wait for one set only)
  const int r0 = it.z0 - 2;
  const int rlo = wall ? max(r0, 0) : r0;
  const int rhi = wall ? min(it.z1 + 1, N - 1) : it.z1 + 1;
  auto clampr = [&](int r) { return r < rlo ? rlo : (r > rhi ? rhi : r); };
  fetch(preA, clampr(r0));
  fetch(preB, clampr(r0 + 1));
  T wM[3] = {};   // slot m: in-plane maximum of q on plane r-3+m
  // iteration r: plane r (in cur) to its ring slot, plane r+2 into cur
  auto body = [&](int r, T (&cur)[I2::NPER]) {
    if (valid(r)) {
      T* __restrict__ dst = sT[wrapm(r, 4)];
#pragma unroll
      for (int i = 0; i < I2::NPER; ++i) dst[(int)threadIdx.x + i * NT] = cur[i];
    }
    fetch(cur, clampr(r + 2));
    __syncthreads();
    const int p = r - 1;
    T m = T(0);
    if (r >= it.z0 && valid(p)) {
      const T* A = sT[wrapm(p, 4)];
      const T* Am = sT[wrapm(p - 1, 4)];
      const T* Ap = sT[wrapm(p + 1, 4)];
      const bool zok = valid(p - 1) && valid(p + 1);
      for (int t = threadIdx.x; t < P1::N; t += NT) {
        const int yy = t / P1::W, xx = t - yy * P1::W;
        const int x = xx - 1, y = yy - 1;
        const T v = A[P2::at(x, y)];
        T d2 = fabs(A[P2::at(x + 1, y)] - T(2) * v + A[P2::at(x - 1, y)]) +
               fabs(A[P2::at(x, y + 1)] - T(2) * v + A[P2::at(x, y - 1)]);
        if (zok) d2 = d2 + fabs(Ap[P2::at(x, y)] - T(2) * v + Am[P2::at(x, y)]);
        const T den = fabs(v) + d2 / ph.q_max;
        sQ[t] = den > T(0) ? d2 / den : T(0);
      }
      __syncthreads();
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) m = fmax(m, sQ[P1::at(tx + dx, ty + dy)]);
    }
    push(wM, m);
    const int oz = r - 2;
    if (own && oz >= it.z0 && oz < it.z1 && valid(oz)) {
      const T mz = fmax(fmax(wM[0], wM[1]), wM[2]);
      const T fac = mz < ph.q_lim ? mz : ph.q_lim;
      tout[col(oz)] = sT[wrapm(oz, 4)][P2::at(tx, ty)] * fac;
    }
  };
  for (int r = r0; r <= it.z1 + 1; r += 2) {
    body(r, preA);
    if (r + 1 <= it.z1 + 1) body(r + 1, preB);
  }
  ZLOOP_END
}

// ln <e_m> over each z plane of every box (eq. ediffav).  e_m = e / rho is
// summed in float64 in a fixed order (deterministic): k_plane_sum gives
// workgroup (P, s) the s-th of kPlaneSlices contiguous slices of plane P
// (planes of all boxes back to back, BoxDev::poff); k_plane_lnmean adds the
// slices of each plane in order and writes the log of the mean.

template <class T>
__global__ __launch_bounds__(256) void k_plane_sum(const BoxDev* __restrict__ boxes, int nbox,
                                                   const T* __restrict__ rho, const T* __restrict__ e,
                                                   double* __restrict__ part) {
  // rho == nullptr: sum e itself (for the plane means of P)
  __shared__ double sh[256];
  const int P = (int)blockIdx.x / kPlaneSlices, sl = (int)blockIdx.x % kPlaneSlices;
  int bi = 0;
  while (bi + 1 < nbox && boxes[bi + 1].poff <= P) ++bi;
  const BoxDev b = boxes[bi];
  const int n = b.nx * b.ny;
  const int i0 = (int)((long long)n * sl / kPlaneSlices), i1 = (int)((long long)n * (sl + 1) / kPlaneSlices);
  const long long base = b.off + (long long)(P - b.poff) * n;
  double s = 0.0;
  if (rho)
    for (int i = i0 + (int)threadIdx.x; i < i1; i += 256) s += (double)e[base + i] / (double)rho[base + i];
  else
    for (int i = i0 + (int)threadIdx.x; i < i1; i += 256) s += (double)e[base + i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

template <class T>
__global__ __launch_bounds__(256) void k_plane_lnmean(const BoxDev* __restrict__ boxes, int nbox,
                                                      int nplanes, const double* __restrict__ part,
                                                      double scale, T* __restrict__ out) {
  const int P = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (P >= nplanes) return;
  int bi = 0;
  while (bi + 1 < nbox && boxes[bi + 1].poff <= P) ++bi;
  double s = 0.0;
  for (int sl = 0; sl < kPlaneSlices; ++sl) s += part[P * kPlaneSlices + sl];
  out[P] = T(log(scale * s / ((double)boxes[bi].nx * boxes[bi].ny)));
}

// Courant time step of the current state from the per-item maxima of A1 / A2
// (eq. courantcond, wave and diffusion limits), into dt_dev[0].
__global__ __launch_bounds__(256) void k_dt(const BoxDev* __restrict__ boxes,
                                            const ZItem* __restrict__ items, int nitems,
                                            const CPart* __restrict__ cpart, double Cdt,
                                            double Cdtd, double nuB, double eta_const,
                                            double* __restrict__ dt_dev) {
  __shared__ double sh[256];
  double best = 1e300;
  for (int i = threadIdx.x; i < nitems; i += 256) {
    const BoxDev b = boxes[items[i].box];
    const double h = b.hmin, ratio = b.hmax / b.hmin;
    const double cm = cpart[i].cmax, nm = cpart[i].numax;
    const double eta_speed = eta_const > 0.0 ? eta_const / h : nuB * nm;
    const double dm = fmax(nm, eta_speed * ratio);
    if (cm > 0.0) best = fmin(best, Cdt * h / cm);
    if (dm > 0.0) best = fmin(best, Cdtd * h / dm);
  }
  sh[threadIdx.x] = best;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) dt_dev[0] = sh[0];
}

// Totals of the per-item partials of mhd_reductions and the three limits of
// eq. courantcond: Cdt h_min / cmax and Cdtd h_min / dmax with each item's
// own box spacing (the smallest over items, with its cell), Cdtr / rmax.
// Each thread folds items t, t + kRedThreads, ... in order; the threads
// combine in a fixed tree, so the result is deterministic.
__device__ __forceinline__ void wave_minarg(double& v, long long& a) {
  for (int o = 32; o > 0; o >>= 1) {
    const double v2 = __shfl_xor(v, o, 64);
    const long long a2 = __shfl_xor(a, o, 64);
    if (v2 < v || (v2 == v && a2 < a)) {
      v = v2;
      a = a2;
    }
  }
}

constexpr int kRedThreads = 256;
__global__ __launch_bounds__(kRedThreads) void k_red_final(const BoxDev* __restrict__ boxes,
                                                    const ZItem* __restrict__ items, int nitems,
                                                    const RedItem* __restrict__ red, double Cdt,
                                                    double Cdtd, double Cdtr, RedTotal* __restrict__ out) {
  constexpr long long NOARG = 0x7fffffffffffffffLL;
  const double inf = __builtin_huge_val();
  double s[8] = {}, mx[3] = {}, c = 0.0, d = 0.0, r = 0.0, tw = inf, td = inf;
  long long ca = NOARG, da = NOARG, ra = NOARG, wa = NOARG, dda = NOARG, nf = 0, np = 0;
  for (int i = threadIdx.x; i < nitems; i += kRedThreads) {
    const RedItem& R = red[i];
    const BoxDev& b = boxes[items[i].box];
    for (int q = 0; q < 8; ++q) s[q] += R.sum[q];
    for (int q = 0; q < 3; ++q) mx[q] = fmax(mx[q], R.mx[q]);
    if (R.cmax > c || (R.cmax == c && R.carg < ca)) { c = R.cmax; ca = R.carg; }
    if (R.dmax > d || (R.dmax == d && R.darg < da)) { d = R.dmax; da = R.darg; }
    if (R.rmax > r || (R.rmax == r && R.rarg < ra)) { r = R.rmax; ra = R.rarg; }
    const double w = R.cmax > 0.0 ? Cdt * b.hmin / R.cmax : inf;
    const double dd = R.dmax > 0.0 ? Cdtd * b.hmin / R.dmax : inf;
    if (w < tw || (w == tw && R.carg < wa)) { tw = w; wa = R.carg; }
    if (dd < td || (dd == td && R.darg < dda)) { td = dd; dda = R.darg; }
    nf += R.nonfinite;
    np += R.nonpositive;
  }
  for (int q = 0; q < 8; ++q) s[q] = wave_sum(s[q]);
  for (int q = 0; q < 3; ++q) mx[q] = wave_max(mx[q]);
  wave_maxarg(c, ca);
  wave_maxarg(d, da);
  wave_maxarg(r, ra);
  wave_minarg(tw, wa);
  wave_minarg(td, dda);
  nf = wave_isum(nf);
  np = wave_isum(np);
  __shared__ double sd[kRedThreads / 64][16];
  __shared__ long long sl[kRedThreads / 64][7];
  const int w = (int)threadIdx.x / 64;
  if (threadIdx.x % 64 == 0) {
    for (int q = 0; q < 8; ++q) sd[w][q] = s[q];
    for (int q = 0; q < 3; ++q) sd[w][8 + q] = mx[q];
    sd[w][11] = c;
    sd[w][12] = d;
    sd[w][13] = r;
    sd[w][14] = tw;
    sd[w][15] = td;
    sl[w][0] = ca;
    sl[w][1] = da;
    sl[w][2] = ra;
    sl[w][3] = wa;
    sl[w][4] = dda;
    sl[w][5] = nf;
    sl[w][6] = np;
  }
  __syncthreads();
  // the waves in order: thread q < 8 adds sum q; thread 8 the rest
  if (threadIdx.x < 8) {
    double v = 0.0;
    for (int x = 0; x < kRedThreads / 64; ++x) v += sd[x][threadIdx.x];
    out->sum[threadIdx.x] = v;
  } else if (threadIdx.x == 8) {
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, cm = 0.0, dm = 0.0, rm = 0.0, dw = inf, dd = inf;
    long long xa = NOARG, ra_ = NOARG, wa_ = NOARG, da_ = NOARG, nf_ = 0, np_ = 0;
    for (int x = 0; x < kRedThreads / 64; ++x) {
      m0 = fmax(m0, sd[x][8]);
      m1 = fmax(m1, sd[x][9]);
      m2 = fmax(m2, sd[x][10]);
      if (sd[x][11] > cm || (sd[x][11] == cm && sl[x][0] < xa)) { cm = sd[x][11]; xa = sl[x][0]; }
      dm = fmax(dm, sd[x][12]);
      if (sd[x][13] > rm || (sd[x][13] == rm && sl[x][2] < ra_)) { rm = sd[x][13]; ra_ = sl[x][2]; }
      if (sd[x][14] < dw || (sd[x][14] == dw && sl[x][3] < wa_)) { dw = sd[x][14]; wa_ = sl[x][3]; }
      if (sd[x][15] < dd || (sd[x][15] == dd && sl[x][4] < da_)) { dd = sd[x][15]; da_ = sl[x][4]; }
      nf_ += sl[x][5];
      np_ += sl[x][6];
    }
    out->mx[0] = m0;
    out->mx[1] = m1;
    out->mx[2] = m2;
    out->cmax = cm;
    out->dmax = dm;
    out->rmax = rm;
    out->dtw = dw;
    out->dtd = dd;
    out->dtr = rm > 0.0 ? Cdtr / rm : inf;
    out->warg = wa_;
    out->darg = da_;
    out->rarg = ra_;
    out->nonfinite = nf_;
    out->nonpositive = np_;
  }
}

template <class T, int TX, int TY>
static void launch_zreduce_t(const ZLaunch& L, CP8<T> f, CP8<T> dfdt, const ZWork<T>& w, const Phys<T>& ph,
                             const T* ztab, RedItem* red, double nuB, double eta_const) {
  const int n = L.nitems;
  const dim3 grid(8 * ((n + 7) / 8)), block(TX * TY);
  if (smag_on(ph)) {
    hipLaunchKernelGGL((zA1<T, TX, TY, false, true, true>), grid, block, 0, L.stream, L.boxes, L.items, n, ztab,
                       (int*)nullptr, f, ph, w, (CPart*)nullptr, dfdt, red);
    hipLaunchKernelGGL((zS<T, TX, TY, false>), grid, block, 0, L.stream, L.boxes, L.items, n, ztab,
                       (int*)nullptr, ph, w);
  } else {
    hipLaunchKernelGGL((zA1<T, TX, TY, false, true>), grid, block, 0, L.stream, L.boxes, L.items, n, ztab,
                       (int*)nullptr, f, ph, w, (CPart*)nullptr, dfdt, red);
  }
  if (ph.terms & T_MAX5)
    hipLaunchKernelGGL((zA2<T, TX, TY, false, true, 5>), grid, block, 0, L.stream, L.boxes, L.items, n, ztab,
                       (int*)nullptr, w, (CPart*)nullptr, nuB, eta_const, red);
  else
    hipLaunchKernelGGL((zA2<T, TX, TY, false, true>), grid, block, 0, L.stream, L.boxes, L.items, n, ztab,
                       (int*)nullptr, w, (CPart*)nullptr, nuB, eta_const, red);
}

template <class T>
void launch_zreduce(const ZLaunch& L, CP8<T> f, CP8<T> dfdt, const ZWork<T>& w, const Phys<T>& ph,
                    const T* ztab, RedItem* red, RedTotal* tot, double Cdt, double Cdtd, double Cdtr,
                    double nuB, double eta_const) {
  switch (L.tile) {
    case ZTILE_32x8: launch_zreduce_t<T, 32, 8>(L, f, dfdt, w, ph, ztab, red, nuB, eta_const); break;
    case ZTILE_16x16: launch_zreduce_t<T, 16, 16>(L, f, dfdt, w, ph, ztab, red, nuB, eta_const); break;
    case ZTILE_16x8: launch_zreduce_t<T, 16, 8>(L, f, dfdt, w, ph, ztab, red, nuB, eta_const); break;
    case ZTILE_64x8: launch_zreduce_t<T, 64, 8>(L, f, dfdt, w, ph, ztab, red, nuB, eta_const); break;
    case ZTILE_32x16: launch_zreduce_t<T, 32, 16>(L, f, dfdt, w, ph, ztab, red, nuB, eta_const); break;
    default: launch_zreduce_t<T, 64, 4>(L, f, dfdt, w, ph, ztab, red, nuB, eta_const); break;
  }
  hipLaunchKernelGGL(k_red_final, dim3(1), dim3(kRedThreads), 0, L.stream, L.boxes, L.items, L.nitems, red, Cdt, Cdtd,
                     Cdtr, tot);
}

template void launch_zreduce<float>(const ZLaunch&, CP8<float>, CP8<float>, const ZWork<float>&,
                                    const Phys<float>&, const float*, RedItem*, RedTotal*, double, double,
                                    double, double, double);
template void launch_zreduce<double>(const ZLaunch&, CP8<double>, CP8<double>, const ZWork<double>&,
                                     const Phys<double>&, const double*, RedItem*, RedTotal*, double, double,
                                     double, double, double);

__global__ __launch_bounds__(128) void k_qreset(int* q) {
  if ((int)threadIdx.x < kQueueInts) q[threadIdx.x] = 0;
}

template <class T, int TX, int TY, bool PERS>
static void launch_zstage_m(const ZLaunch& L, const ZStageArgs<T>& a) {
  const int n = L.nitems;
  const dim3 block(TX * TY);
  int* q = PERS ? L.queue : nullptr;
  auto grid = [&](const void* kern) {
    if (!q) return dim3(8 * ((n + 7) / 8));
    const int r = std::min(n, zresident_groups(kern, TX * TY, L.ncu));
    return dim3(std::max(8, r - r % 8));
  };
  if (q) hipLaunchKernelGGL(k_qreset, dim3(1), dim3(128), 0, L.stream, q);
  L.at(PASS_PRIM);
  if (smag_on(a.ph)) {
    hipLaunchKernelGGL((zA1<T, TX, TY, PERS, false, true>), grid((const void*)zA1<T, TX, TY, PERS, false, true>),
                       block, 0, L.stream, L.boxes, L.items, n, a.ztab, q, a.f, a.ph, a.w, a.cpart);
    hipLaunchKernelGGL((zS<T, TX, TY, PERS>), grid((const void*)zS<T, TX, TY, PERS>), block, 0, L.stream,
                       L.boxes, L.items, n, a.ztab, q ? q + 64 : q, a.ph, a.w);
  } else {
    hipLaunchKernelGGL((zA1<T, TX, TY, PERS>), grid((const void*)zA1<T, TX, TY, PERS>), block, 0, L.stream,
                       L.boxes, L.items, n, a.ztab, q, a.f, a.ph, a.w, a.cpart);
  }
  L.at(PASS_MEAN3);
  if (a.ph.terms & T_MAX5)
    hipLaunchKernelGGL((zA2<T, TX, TY, PERS, false, 5>), grid((const void*)zA2<T, TX, TY, PERS, false, 5>), block,
                       0, L.stream, L.boxes, L.items, n, a.ztab, q ? q + 8 : q, a.w, a.cpart);
  else
    hipLaunchKernelGGL((zA2<T, TX, TY, PERS>), grid((const void*)zA2<T, TX, TY, PERS>), block, 0, L.stream,
                       L.boxes, L.items, n, a.ztab, q ? q + 8 : q, a.w, a.cpart);
  if (a.cpart) {
    L.at(PASS_REDUCE);
    hipLaunchKernelGGL(k_dt, dim3(1), dim3(256), 0, L.stream, L.boxes, L.items, n, a.cpart, a.Cdt,
                       a.Cdtd, a.nuB, a.eta_const, a.dt_dev);
    L.at(PASS_MEAN3);   // the plane means below are booked with A2 in every stage
  }
  if ((a.ph.terms & T_EDIFF) && (a.ph.terms & T_EDIFFAV)) {
    hipLaunchKernelGGL(k_plane_sum<T>, dim3(L.nplanes * kPlaneSlices), dim3(256), 0, L.stream, L.boxes, L.nbox,
                       a.f.p[0], a.f.p[4], a.lnpart);
    hipLaunchKernelGGL(k_plane_lnmean<T>, dim3((L.nplanes + 255) / 256), dim3(256), 0, L.stream, L.boxes,
                       L.nbox, L.nplanes, a.lnpart, 1.0, a.lnavg);
  }
  const bool lnp = (a.ph.terms & T_PRES) && (a.ph.terms & T_LNP);
  if (lnp) {   // ln P_aver, P = (gamma - 1) e
    hipLaunchKernelGGL(k_plane_sum<T>, dim3(L.nplanes * kPlaneSlices), dim3(256), 0, L.stream, L.boxes, L.nbox,
                       (const T*)nullptr, a.f.p[4], a.lnpart);
    hipLaunchKernelGGL(k_plane_lnmean<T>, dim3((L.nplanes + 255) / 256), dim3(256), 0, L.stream, L.boxes,
                       L.nbox, L.nplanes, a.lnpart, (double)a.ph.gamma1, a.w.lnpav);
  }
  L.at(PASS_EDGES);
  // the optional passes run in grid mode (their own launches, no queue)
  const dim3 gq(8 * ((n + 7) / 8));
  // second-order switch: the flags of every cell; pass P then writes the
  // second-order div u that pass Q's tau_zz takes, so P goes first
  ZWork<T> wq = a.w;
  const bool o2 = (a.ph.terms & T_ORDER2) && (a.ph.terms & T_VISC);
  if (o2) {
    hipLaunchKernelGGL((zRough<T, TX, TY, false>), gq, block, 0, L.stream, L.boxes, L.items, n, a.ztab,
                       (int*)nullptr, a.f, a.ph, a.w);
    wq.rgh = a.w.arr(WS_RGH);
  }
  // quenching: the raw stress (stress-only launches of P and Q), then its
  // quenched version, which P and Q below take in place of their own
  if ((a.ph.terms & T_QUENCH) && (a.ph.terms & T_VISC)) {
    hipLaunchKernelGGL((zP<T, TX, TY, false, true>), gq, block, 0, L.stream, L.boxes, L.items, n, a.ztab,
                       (int*)nullptr, a.f, a.ph, wq);
    hipLaunchKernelGGL((zQ<T, TX, TY, false, QM_EDGES | QM_TAU>), gq, block, 0, L.stream, L.boxes, L.items, n,
                       a.ztab, (int*)nullptr, a.f, a.ph, wq, a.lnavg, a.w.lnpav);
    hipLaunchKernelGGL((zQ<T, TX, TY, false, QM_ZC | QM_TAU>), gq, block, 0, L.stream, L.boxes, L.items, n,
                       a.ztab, (int*)nullptr, a.f, a.ph, wq, a.lnavg, a.w.lnpav);
    hipLaunchKernelGGL((zQn<T, TX, TY>), dim3(gq.x, TAU_COUNT), block, 0, L.stream, L.boxes, L.items, n, a.ztab,
                       a.ph, a.w);
    wq.tq = a.w.arr(WS_TQ0);
  }
  auto launch_p = [&]() {
    L.at(PASS_CF);
    hipLaunchKernelGGL((zP<T, TX, TY, PERS>), grid((const void*)zP<T, TX, TY, PERS>), block, 0, L.stream,
                       L.boxes, L.items, n, a.ztab, q ? q + 24 : q, a.f, a.ph, wq);
  };
  if (o2) {
    launch_p();
    L.at(PASS_EDGES);
  }
  hipLaunchKernelGGL((zQ<T, TX, TY, PERS, QM_EDGES>), grid((const void*)zQ<T, TX, TY, PERS, QM_EDGES>), block, 0,
                     L.stream, L.boxes, L.items, n, a.ztab, q ? q + 16 : q, a.f, a.ph, wq, a.lnavg,
                     a.w.lnpav);
  if (lnp)
    hipLaunchKernelGGL((zQ<T, TX, TY, PERS, QM_ZC | QM_LNP>), grid((const void*)zQ<T, TX, TY, PERS, QM_ZC | QM_LNP>),
                       block, 0, L.stream, L.boxes, L.items, n, a.ztab, q ? q + 32 + 8 * kNFMasks : q, a.f, a.ph,
                       wq, a.lnavg, a.w.lnpav);
  else
    hipLaunchKernelGGL((zQ<T, TX, TY, PERS, QM_ZC>), grid((const void*)zQ<T, TX, TY, PERS, QM_ZC>), block, 0,
                       L.stream, L.boxes, L.items, n, a.ztab, q ? q + 32 + 8 * kNFMasks : q, a.f, a.ph, wq,
                       a.lnavg, a.w.lnpav);
  if (!o2) launch_p();
  L.at(PASS_FINAL);
  launch_final<T, PERS>(L, a, q);
  L.at(PASS_END);
}

template <class T, int TX, int TY>
static void launch_zstage_t(const ZLaunch& L, const ZStageArgs<T>& a) {
  if (L.persistent) launch_zstage_m<T, TX, TY, true>(L, a);
  else launch_zstage_m<T, TX, TY, false>(L, a);
}

template <class T>
void launch_zstage(const ZLaunch& L, const ZStageArgs<T>& a) {
  switch (L.tile) {
    case ZTILE_32x8: launch_zstage_t<T, 32, 8>(L, a); break;
    case ZTILE_16x16: launch_zstage_t<T, 16, 16>(L, a); break;
    case ZTILE_16x8: launch_zstage_t<T, 16, 8>(L, a); break;
    case ZTILE_64x8: launch_zstage_t<T, 64, 8>(L, a); break;
    case ZTILE_32x16: launch_zstage_t<T, 32, 16>(L, a); break;
    default:
      launch_zstage_t<T, 64, 4>(L, a);
      break;
  }
}

template void launch_zstage<float>(const ZLaunch&, const ZStageArgs<float>&);
template void launch_zstage<double>(const ZLaunch&, const ZStageArgs<double>&);

}  // namespace smhd
