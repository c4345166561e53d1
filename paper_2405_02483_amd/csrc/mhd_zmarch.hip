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
  (void)zt;

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
template <class T, int TX, int TY, bool PERS, bool RED = false>
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
  for (int r = it.z0 - 5; r <= it.z1 + 4; ++r) {
    T rr = T(0), pz = T(0), e = T(0), bz = T(0);
    T ubx = T(0), uby = T(0), bbx = T(0), bby = T(0), dxy = T(0), dxb = T(0);
    if (valid(r)) {
      const int k = kk(r);
      __syncthreads();
      load_plane(sR, f.p[0], b, i5, k);
      load_plane(sPX, f.p[1], b, i3, k);
      load_plane(sPY, f.p[2], b, i3, k);
      load_plane(sBX, f.p[5], b, i3, k);
      load_plane(sBY, f.p[6], b, i3, k);
      __syncthreads();
      const long long o = col(r);
      rr = sR[PR::at(tx, ty)];
      pz = f.p[3][o];
      e = f.p[4][o];
      bz = f.p[7][o];
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
        rs[0] += rd;
        rs[1] += pxd;
        rs[2] += pyd;
        rs[3] += pzd;
        rs[4] += 0.5 * (pxd * uxd + pyd * uyd);
        rs[5] += bxd * bxd + byd * byd + bzd * bzd;
        rs[6] += ed;
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
        rs[4] += 0.5 * (double)fPZ[0] * (double)uzq;
        rum = fmax(rum, fabs((double)uzq));
      }
    }
    push(wUZ, uzq);                       // wUZ slot m = plane r-7+m
    // centre quantities of plane q = r - 5
    const int q = r - 5;
    if (valid(q) && q >= it.z0 && q < it.z1) {
      const T ubz = zwin<0, 1, 6, 2>(wUZ, q, wall, N, T(0), zt);
      const T dzz = zwin<1, 1, 6, 2>(wUZ, q, wall, N, g.hzi, zt);
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
        nus = ph.nu1 * norm3(fUBX[0], fUBY[0], ubz) + ph.nu3 * (cs + ca) + ph.nu2 * g.h * relu;
      }
      if (own) {
        const long long o = col(q);
        nus_out[o] = nus;
        D_out[o] = D;
        if (divb) divb_out[o] = fDXB[0] + zwin<1, 1, 8, 2>(wBZ, q, wall, N, g.hzi, zt);
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
            const double db = (double)fDXB[0] + (double)zwin<1, 1, 8, 2>(wBZ, q, wall, N, g.hzi, zt);
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
// A2: m = max over the 3x3x3 neighbourhood (x, y through LDS; z over a ring
// of three x/y-maximum planes), then three-cell means along x, y (LDS) and
// z (register window), floor 1e-30, and ln.
//
// RED (the reduction instantiation of mhd_reductions): also the diffusion
// speed max(<nu>, eta_speed h_max / h_min) of eq. courantcond, eta_speed =
// nuB <nu> or eta_const / h_min, and its first maximal cell, into red[item].
template <class T, int TX, int TY, bool PERS, bool RED = false>
__global__ __launch_bounds__(TX * TY) void zA2(const BoxDev* __restrict__ boxes,
                                               const ZItem* __restrict__ items, int nitems, const T* __restrict__ ztab,
                                               int* __restrict__ queue,
                                               ZWork<T> ws, CPart* __restrict__ cpart,
                                               double nuB = 0.0, double eta_const = 0.0,
                                               RedItem* __restrict__ red = nullptr) {
  const T* __restrict__ nus = ws.arr(WS_NUS);
  T* __restrict__ lnt_out = ws.arr(WS_LNT);
  using PN = Plane<TX, TY, 2>;
  using PM = Plane<TX, TY, 1>;
  constexpr int NT = TX * TY;
  __shared__ T sN[PN::NP];
  __shared__ T sMX[3][PM::NP];
  __shared__ T sM[PM::NP];
  __shared__ double sred[NT];
  ZLOOP_BEGIN
  PlaneIdx<TX, TY, 2> i2;
  i2.init(b, it.x0, it.y0);
  T wS[3] = {};
  double numax = 0.0;
  double rd = 0.0;
  long long rda = 0x7fffffffffffffffLL;
  for (int r = it.z0 - 2; r <= it.z1 + 1; ++r) {
    if (valid(r)) {
      __syncthreads();
      load_plane(sN, nus, b, i2, kk(r));
      __syncthreads();
      T* dst = sMX[wrapm(r, 3)];
      for (int t = threadIdx.x; t < PM::N; t += NT) {
        const int yy = t / PM::W, xx = t - yy * PM::W;
        const int x = xx - 1, y = yy - 1;
        T m = sN[PN::at(x, y)];
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) m = fmax(m, sN[PN::at(x + dx, y + dy)]);
        dst[t] = m;
      }
    }
    const int q1 = r - 1;
    T sxy = T(0);
    if (valid(q1)) {
      __syncthreads();
      const bool lo = valid(q1 - 1), hi = valid(q1 + 1);
      const T* a = sMX[wrapm(q1, 3)];
      const T* am = sMX[wrapm(q1 - 1, 3)];
      const T* ap = sMX[wrapm(q1 + 1, 3)];
      for (int t = threadIdx.x; t < PM::N; t += NT) {
        T m = a[t];
        if (lo) m = fmax(m, am[t]);
        if (hi) m = fmax(m, ap[t]);
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
    push(wS, sxy);                        // wS slot m = plane r-3+m
    const int q = r - 2;
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
  constexpr bool kE = QM & QM_EDGES, kZ = QM & QM_ZC;
  constexpr int NPL = kE ? P3::NP : 1;
  __shared__ T sR[NPL], sL[NPL];
  __shared__ T sUZ[3][NPL], sBZ[3][NPL], sPZ[3][NPL];
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
  for (int r = it.z0 - 3; r <= it.z1 + 2; ++r) {
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
        load_plane(sUZ[sl], uzg, b, i3, k);
        load_plane(sBZ[sl], f.p[7], b, i3, k);
        load_plane(sPZ[sl], f.p[3], b, i3, k);
        __syncthreads();
        rx = op6<0, 0, T>([&](int m) { return sR[P3::at(tx + m, ty)]; }, T(0));
        ry = op6<0, 0, T>([&](int m) { return sR[P3::at(tx, ty + m)]; }, T(0));
        lx = op6<0, 0, T>([&](int m) { return sL[P3::at(tx + m, ty)]; }, T(0));
        ly = op6<0, 0, T>([&](int m) { return sL[P3::at(tx, ty + m)]; }, T(0));
        px = f.p[1][o];
        py = f.p[2][o];
        ux = px / rx;
        uy = py / ry;
        bxv = f.p[5][o];
        byv = f.p[6][o];
      }
      if constexpr (kZ) {
        // own column only: from LDS when the planes are there
        if constexpr (kE) {
          pzv = sPZ[sl][P3::at(tx, ty)];
          uzv = sUZ[sl][P3::at(tx, ty)];
          rhov = sR[P3::at(tx, ty)];
          nuv = exp(sL[P3::at(tx, ty)]);
        } else {
          pzv = f.p[3][o];
          uzv = uzg[o];
          rhov = f.p[0][o];
          nuv = exp(lntg[o]);
        }
        ev = f.p[4][o];
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
      // ---- y-edge
      if constexpr (kE) {
        const T zRX = zwin<0, 0, 6, 3>(wRX, q, wall, N, T(0), zt);
        const T zPX = zwin<0, 0, 6, 3>(wPX, q, wall, N, T(0), zt);
        const T zUX = zwin<0, 0, 6, 3>(wUX, q, wall, N, T(0), zt);
        const T dzUX = zwin<1, 0, 6, 3>(wUX, q, wall, N, g.hzi, zt);
        const T zBX = zwin<0, 0, 6, 3>(wBX, q, wall, N, T(0), zt);
        const T dzBX = zwin<1, 0, 6, 3>(wBX, q, wall, N, g.hzi, zt);
        const T xUZ = op6<0, 0, T>([&](int m) { return UZ[P3::at(tx + m, ty)]; }, T(0));
        const T dxUZ = op6<1, 0, T>([&](int m) { return UZ[P3::at(tx + m, ty)]; }, g.hxi);
        const T xBZ = op6<0, 0, T>([&](int m) { return BZ[P3::at(tx + m, ty)]; }, T(0));
        const T dxBZ = op6<1, 0, T>([&](int m) { return BZ[P3::at(tx + m, ty)]; }, g.hxi);
        const T xPZ = op6<0, 0, T>([&](int m) { return PZ[P3::at(tx + m, ty)]; }, T(0));
        T nxz = T(0), txz = T(0), sxz = T(0);
        if (need_nu) nxz = g.lxz * exp(zwin<0, 0, 6, 3>(wLX, q, wall, N, T(0), zt));
        if (visc) {
          sxz = T(0.5) * (dzUX + dxUZ);
          txz = zRX * nxz * sxz;
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
      if constexpr (kE) {
        const T zRY = zwin<0, 0, 6, 3>(wRY, q, wall, N, T(0), zt);
        const T zPY = zwin<0, 0, 6, 3>(wPY, q, wall, N, T(0), zt);
        const T zUY = zwin<0, 0, 6, 3>(wUY, q, wall, N, T(0), zt);
        const T dzUY = zwin<1, 0, 6, 3>(wUY, q, wall, N, g.hzi, zt);
        const T zBY = zwin<0, 0, 6, 3>(wBY, q, wall, N, T(0), zt);
        const T dzBY = zwin<1, 0, 6, 3>(wBY, q, wall, N, g.hzi, zt);
        const T yUZ = op6<0, 0, T>([&](int m) { return UZ[P3::at(tx, ty + m)]; }, T(0));
        const T dyUZ = op6<1, 0, T>([&](int m) { return UZ[P3::at(tx, ty + m)]; }, g.hyi);
        const T yBZ = op6<0, 0, T>([&](int m) { return BZ[P3::at(tx, ty + m)]; }, T(0));
        const T dyBZ = op6<1, 0, T>([&](int m) { return BZ[P3::at(tx, ty + m)]; }, g.hyi);
        const T yPZ = op6<0, 0, T>([&](int m) { return PZ[P3::at(tx, ty + m)]; }, T(0));
        T nyz = T(0), tyz = T(0), syz = T(0);
        if (need_nu) nyz = g.lyz * exp(zwin<0, 0, 6, 3>(wLY, q, wall, N, T(0), zt));
        if (visc) {
          syz = T(0.5) * (dzUY + dyUZ);
          tyz = zRY * nyz * syz;
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
      if constexpr (kZ) {
        T hz = T(0);
        if (adv) hz = -zwin<0, 0, 6, 3>(wE, q, wall, N, T(0), zt) * wUZ[3];
        if (ediff)
          hz = hz + ph.nuE * zwin<0, 0, 6, 3>(wRho, q, wall, N, T(0), zt) *
                        (g.lz * zwin<0, 0, 6, 3>(wNu, q, wall, N, T(0), zt)) *
                        zwin<0, 0, 6, 3>(wEm, q, wall, N, T(0), zt) *
                        zwin<1, 0, 6, 3>(wLem, q, wall, N, g.hzi, zt);
        if (own) {
          ws.q(QOUT_HZ)[o] = hz;
          // pressure gradient on its own: folded into the flux, a pressure
          // of order one would swamp the much smaller stresses in float32
          T dpz = T(0);
          if (pres) {
            if constexpr (kL)
              dpz = exp(zwin<0, 0, 6, 3>(wLpa, q, wall, N, T(0), zt)) *
                    exp(zwin<0, 0, 6, 3>(wLq, q, wall, N, T(0), zt)) *
                    (zwin<1, 0, 6, 3>(wLq, q, wall, N, g.hzi, zt) +
                     zwin<1, 0, 6, 3>(wLpa, q, wall, N, g.hzi, zt));
            else
              dpz = ph.gamma1 * zwin<1, 0, 6, 3>(wE, q, wall, N, g.hzi, zt);
          }
          ws.q(QOUT_DPZ)[o] = dpz;
        }
      }
    }
    // centre terms of plane q2 = r - 3 (window slot 2)
    const int q2 = r - 3;
    if (kZ && valid(q2) && q2 >= it.z0 && q2 < it.z1) {
      const long long o = col(q2);
      const T szz = zwin<1, 1, 6, 2>(wUZ, q2, wall, N, g.hzi, zt);
      T gzz = T(0), czz = T(0);
      if (visc) {
        const T tzz = wRho[2] * (g.lz * wNu[2]) * (szz + ph.c1 * Dg[o]);
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
// Lyz, Qz (as in Q), the centre terms Gxx = tau_xx - xup(p_x) xup(u_x) - P,
// Gyy, Qc = tau_xx S_xx + tau_yy S_yy - P div u, and the x/y-face energy
// fluxes Hx, Hy (eq. ien, eq. ediffuse).
template <class T, int TX, int TY, bool PERS>
__global__ __launch_bounds__(TX * TY) void zP(const BoxDev* __restrict__ boxes,
                                              const ZItem* __restrict__ items, int nitems, const T* __restrict__ ztab,
                                               int* __restrict__ queue,
                                              CP8<T> f, Phys<T> ph, ZWork<T> ws) {
  const T* __restrict__ lntg = ws.arr(WS_LNT);
  const T* __restrict__ Dg = ws.arr(WS_D);
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
  const bool visc = tm & T_VISC, res = tm & T_RESIST, ind = tm & T_INDUCT, lor = tm & T_LORENTZ,
             adv = tm & T_ADV, pres = tm & T_PRES, ediff = tm & T_EDIFF;
  const bool need_nu = visc || (res && !(ph.eta_const > T(0)));
  const T inv_mu = ph.inv_mu;
  auto S = [&](int q, int x, int y) -> T& { return s3[q * P3::NP + P3::at(x, y)]; };
  for (int k = it.z0; k < it.z1; ++k) {
    __syncthreads();
    load_plane(sR, f.p[0], b, i6, k);
    load_plane(&S(0, -3, -3), f.p[1], b, i3, k);
    load_plane(&S(1, -3, -3), f.p[2], b, i3, k);
    load_plane(&S(2, -3, -3), f.p[4], b, i3, k);
    load_plane(&S(3, -3, -3), f.p[5], b, i3, k);
    load_plane(&S(4, -3, -3), f.p[6], b, i3, k);
    load_plane(&S(5, -3, -3), lntg, b, i3, k);
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
      const T emv = s3[2 * P3::NP + t] / rc;
      s3[9 * P3::NP + t] = emv;
      s3[10 * P3::NP + t] = log(emv);
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
    // ---- z-edge (x-1/2, y-1/2)
    T nxy = T(0), txy = T(0), sxy = T(0);
    if (need_nu)
      nxy = g.lxy * exp(op6<0, 0, T>([&](int m) { return S(13, x, y + m); }, T(0)));
    if (visc) {
      const T rxy = op6<0, 0, T>([&](int m) { return S(11, x, y + m); }, T(0));
      sxy = T(0.5) * (op6<1, 0, T>([&](int m) { return S(6, x, y + m); }, g.hyi) +
                      op6<1, 0, T>([&](int m) { return S(7, x + m, y); }, g.hxi));
      txy = rxy * nxy * sxy;
    }
    const T jz = op6<1, 0, T>([&](int m) { return S(4, x + m, y); }, g.hxi) -
                 op6<1, 0, T>([&](int m) { return S(3, x, y + m); }, g.hyi);
    const T eta = ph.eta_const > T(0) ? ph.eta_const : ph.nuB * nxy;
    const T xBY = op6<0, 0, T>([&](int m) { return S(4, x + m, y); }, T(0));
    const T yBX = op6<0, 0, T>([&](int m) { return S(3, x, y + m); }, T(0));
    const T yUX = op6<0, 0, T>([&](int m) { return S(6, x, y + m); }, T(0));
    const T xUY = op6<0, 0, T>([&](int m) { return S(7, x + m, y); }, T(0));
    T ez = T(0);
    if (ind) ez = ez - (yUX * xBY - xUY * yBX);
    if (res) ez = ez + eta * jz;
    T gxy = txy, gyx = txy;
    if (adv) {
      gxy = gxy - op6<0, 0, T>([&](int m) { return S(0, x, y + m); }, T(0)) * xUY;
      gyx = gyx - op6<0, 0, T>([&](int m) { return S(1, x + m, y); }, T(0)) * yUX;
    }
    T qz = visc ? T(2) * txy * sxy : T(0);
    if (res) qz = qz + eta * jz * jz * inv_mu;
    ws.pq(POUT_GXY)[o] = gxy;
    ws.pq(POUT_GYX)[o] = gyx;
    ws.pq(POUT_EZ)[o] = ez;
    ws.pq(POUT_LXZ)[o] = lor ? jz * xBY : T(0);
    ws.pq(POUT_LYZ)[o] = lor ? jz * yBX : T(0);
    ws.pq(POUT_QZ)[o] = qz;
    // ---- centre
    {
      const T sxx = op6<1, 1, T>([&](int m) { return S(6, x + m, y); }, g.hxi);
      const T syy = op6<1, 1, T>([&](int m) { return S(7, x, y + m); }, g.hyi);
      const T Dc = Dg[o];
      const T Pc = ph.gamma1 * S(2, x, y);
      T gxx = T(0), gyy = T(0), qc = T(0);
      if (visc) {
        const T rn = sR[P6::at(x, y)] * S(8, x, y);
        const T txx = rn * g.lx * (sxx + ph.c1 * Dc);
        const T tyy = rn * g.ly * (syy + ph.c1 * Dc);
        gxx = txx;
        gyy = tyy;
        qc = txx * sxx + tyy * syy;
      }
      if (adv) {
        gxx = gxx - op6<0, 1, T>([&](int m) { return S(0, x + m, y); }, T(0)) *
                        op6<0, 1, T>([&](int m) { return S(6, x + m, y); }, T(0));
        gyy = gyy - op6<0, 1, T>([&](int m) { return S(1, x, y + m); }, T(0)) *
                        op6<0, 1, T>([&](int m) { return S(7, x, y + m); }, T(0));
      }
      if (pres) qc = qc - Pc * Dc;
      ws.pq(POUT_GXX)[o] = gxx;
      ws.pq(POUT_GYY)[o] = gyy;
      ws.pq(POUT_QC)[o] = qc;
      // pressure gradients on the x- and y-faces, kept out of the fluxes
      T dpx = T(0), dpy = T(0);
      if (pres && (tm & T_LNP)) {
        // eq. pressure: exp(ln P_aver) exp(adn(q)) ddadn(q), q = ln(P / P_aver)
        // (the x and y derivatives of the plane mean vanish)
        const T lpa = lnpav[b.poff + k];
        auto lq = [&](int xx, int yy) { return log(ph.gamma1 * S(2, xx, yy)) - lpa; };
        const T epa = exp(lpa);
        dpx = epa * exp(op6<0, 0, T>([&](int m) { return lq(x + m, y); }, T(0))) *
              op6<1, 0, T>([&](int m) { return lq(x + m, y); }, g.hxi);
        dpy = epa * exp(op6<0, 0, T>([&](int m) { return lq(x, y + m); }, T(0))) *
              op6<1, 0, T>([&](int m) { return lq(x, y + m); }, g.hyi);
      } else if (pres) {
        dpx = ph.gamma1 * op6<1, 0, T>([&](int m) { return S(2, x + m, y); }, g.hxi);
        dpy = ph.gamma1 * op6<1, 0, T>([&](int m) { return S(2, x, y + m); }, g.hyi);
      }
      if (tm & T_CORI) {
        // the in-plane parts of the Coriolis force -2 Omega x p (eq. mom),
        // with the sign of a gradient that pass F subtracts: +2 Omega_z p_y
        // on x-faces, -2 Omega_z p_x on y-faces
        dpx -= ph.cor2[2] * op6<0, 0, T>([&](int m) {
                 return op6<0, 1, T>([&](int n) { return S(1, x + m, y + n); }, T(0));
               }, T(0));
        dpy += ph.cor2[2] * op6<0, 0, T>([&](int n) {
                 return op6<0, 1, T>([&](int m) { return S(0, x + m, y + n); }, T(0));
               }, T(0));
      }
      ws.pq(POUT_DPX)[o] = dpx;
      ws.pq(POUT_DPY)[o] = dpy;
    }
    // ---- x- and y-faces: energy fluxes
    {
      T hx = T(0), hy = T(0);
      if (adv) {
        hx = -op6<0, 0, T>([&](int m) { return S(2, x + m, y); }, T(0)) * S(6, x, y);
        hy = -op6<0, 0, T>([&](int m) { return S(2, x, y + m); }, T(0)) * S(7, x, y);
      }
      if (ediff) {
        hx = hx + ph.nuE * S(11, x, y) *
                      (g.lx * op6<0, 0, T>([&](int m) { return S(8, x + m, y); }, T(0))) *
                      op6<0, 0, T>([&](int m) { return S(9, x + m, y); }, T(0)) *
                      op6<1, 0, T>([&](int m) { return S(10, x + m, y); }, g.hxi);
        hy = hy + ph.nuE * S(12, x, y) *
                      (g.ly * op6<0, 0, T>([&](int m) { return S(8, x, y + m); }, T(0))) *
                      op6<0, 0, T>([&](int m) { return S(9, x, y + m); }, T(0)) *
                      op6<1, 0, T>([&](int m) { return S(10, x, y + m); }, g.hyi);
      }
      ws.pq(POUT_HX)[o] = hx;
      ws.pq(POUT_HY)[o] = hy;
    }
  }
  ZLOOP_END
}

// ---------------------------------------------------------------------------
// F: all divergences of P's and Q's quantities and of the momenta, the
// gravity force, wall masking and the RK stage update.  x/y divergences of
// plane r through LDS strips; z divergences scattered into per-thread
// accumulators of output planes r-3..r+3 (first differences for
// derivatives); plane r-3 is then complete.
//
// FM selects the fields this launch completes (bit v: field v); the stage
// runs one launch per mask of kFMasks.  The groups read nearly disjoint
// inputs, and each launch needs a fraction of the registers and LDS.
// Masks: the momenta; rho and e; the magnetic field.
constexpr unsigned kFMasks[] = {0x0Eu, 0x11u, 0xE0u};
constexpr int kNFMasks = sizeof(kFMasks) / sizeof(kFMasks[0]);
// queue counters, 8 per launch: A1, A2, Q edges, P, the F launches, then Q's
// z-face and centre launch
static_assert(32 + 8 * kNFMasks + 8 <= kQueueInts && kQueueInts <= 64, "queue counters per launch");
constexpr bool masks_partition() {
  unsigned all = 0;
  for (unsigned m : kFMasks) {
    if (all & m) return false;
    all |= m;
  }
  return all == 0xFFu;
}
static_assert(masks_partition(), "each field completed by exactly one launch");
template <unsigned FM> __host__ __device__ constexpr bool hasf(int v) { return (FM >> v) & 1u; }
// the field each LDS strip serves, in zF's strip order: x strips, y strips
__host__ __device__ constexpr int kXOwn[9] = {0, 1, 2, 2, 4, 3, 3, 7, 4};
__host__ __device__ constexpr int kYOwn[9] = {0, 1, 1, 2, 4, 3, 3, 7, 4};
// LDS position of strip q among the strips a launch loads (own: kXOwn or
// kYOwn); q = 9 gives their number
template <unsigned FM>
__host__ __device__ constexpr int strip_slot(const int (&own)[9], int q) {
  int n = 0;
  for (int i = 0; i < q; ++i) n += (FM >> own[i]) & 1u;
  return n;
}
__host__ __device__ constexpr int at_least1(int n) { return n > 0 ? n : 1; }

template <class T, int TX, int TY, bool PERS, unsigned FM>
__global__ __launch_bounds__(TX * TY) void zF(const BoxDev* __restrict__ boxes,
                                              const ZItem* __restrict__ items, int nitems, const T* __restrict__ ztab,
                                               int* __restrict__ queue,
                                              CP8<T> f, ZWork<T> ws, Phys<T> ph, P8<T> du,
                                              int du_mode, P8<T> f_out, T alpha, double beta,
                                              const double* __restrict__ dt_dev,
                                              double dt_host) {
  using PXs = Plane<TX, TY, 3, 0>;   // x-halo strips
  using PYs = Plane<TX, TY, 0, 3>;   // y-halo strips
  using P3 = Plane<TX, TY, 3>;
  // x strips: 0 px 1 Gxx 2 Gyx 3 Lyz 4 Hx 5 Gzx 6 Lzy 7 Ey 8 Qy
  // y strips: 0 py 1 Gxy 2 Lxz 3 Gyy 4 Hy 5 Gzy 6 Lzx 7 Ex 8 Qx
  // full:     0 Qz 1 Ez
  // only the strips of this launch's fields occupy LDS
  constexpr bool kQz = hasf<FM>(4), kEz = hasf<FM>(5) || hasf<FM>(6);
  __shared__ T sx[at_least1(strip_slot<FM>(kXOwn, 9)) * PXs::NP];
  __shared__ T sy[at_least1(strip_slot<FM>(kYOwn, 9)) * PYs::NP];
  __shared__ T s2[at_least1(int(kQz) + int(kEz)) * P3::NP];
  // Coriolis force (bit 8 of FM, momentum launch only; its in-plane parts
  // come with pass P's face terms): x strips of px and pz, y strips of py
  // and pz
  constexpr bool kCori = hasf<FM>(8);
  // div B diffusion (B launch): x and y strips of div B
  constexpr bool kDB = hasf<FM>(5);
  __shared__ T sdb[kDB ? PXs::NP + PYs::NP : 1];
  __shared__ T sxc[kCori ? 2 * PXs::NP : 1];
  __shared__ T syc[kCori ? 2 * PYs::NP : 1];
  ZLOOP_BEGIN
  PlaneIdx<TX, TY, 3, 0> ix;
  PlaneIdx<TX, TY, 0, 3> iy;
  PlaneIdx<TX, TY, 3> i3;
  ix.init(b, it.x0, it.y0);
  iy.init(b, it.x0, it.y0);
  i3.init(b, it.x0, it.y0);
  const unsigned tm = ph.terms;
  const bool cont = tm & T_CONT, grav = tm & T_GRAV;
  const T inv_mu = ph.inv_mu;
  const double dt = dt_dev ? *dt_dev : dt_host;
  const T bdt = T(beta * dt);
  // div B diffusion C_divb h^2 / dt grad(div B); absent without a time step
  const T kd = (kDB && dt > 0.0) ? T(double(ph.c_divb) * double(g.h) * double(g.h) / dt) : T(0);
  auto X = [&](int q, int x) -> T { return sx[strip_slot<FM>(kXOwn, q) * PXs::NP + PXs::at(x, ty)]; };
  auto Y = [&](int q, int y) -> T { return sy[strip_slot<FM>(kYOwn, q) * PYs::NP + PYs::at(tx, y)]; };
  auto F2 = [&](int q, int x, int y) -> T { return s2[(q && kQz) * P3::NP + P3::at(x, y)]; };
  auto XC = [&](int q, int x) -> T { return sxc[q * PXs::NP + PXs::at(x, ty)]; };
  auto YC = [&](int q, int y) -> T { return syc[q * PYs::NP + PYs::at(tx, y)]; };
  T acc[7][7];
#pragma unroll
  for (int a = 0; a < 7; ++a)
#pragma unroll
    for (int s = 0; s < 7; ++s) acc[a][s] = T(0);
  // previous-plane values of the z-differentiated quantities (first
  // differences): 0 pz 1 Gxz 2 Gyz 3 Gzz 4 Hz 5 Ey 6 Ex
  T prev[7];
#pragma unroll
  for (int a = 0; a < 7; ++a) prev[a] = T(0);

  // wall masking (Section 10): F vanishes in ghost planes, and for pz also
  // on the two wall faces; Bz evolves on the wall faces
  auto masked = [&](int v, int k, T Fv) -> T {
    if (!wall) return Fv;
    const bool cen = k >= b.g0 && k < b.g1;
    const bool keep = v == 3 ? (k > b.g0 && k < b.g1) : (v == 7 ? (k >= b.g0 && k <= b.g1) : cen);
    return keep ? Fv : T(0);
  };
  // RK stage update of one field at plane k, given its dU and f there
  auto update = [&](int v, long long o, T Fv, T uin, T fin) {
    const T U = (du_mode & DU_READ) ? alpha * uin + Fv : Fv;
    if (du_mode & DU_WRITE) du.p[v][o] = U;
    f_out.p[v][o] = fin + bdt * U;
  };
  // the seven z-accumulated fields at plane k: every load first, so they
  // share one round trip to memory
  auto finalize7 = [&](int k) {
    const long long o = col(k);
    T Fv[7];
#pragma unroll
    for (int a = 0; a < 7; ++a) Fv[a] = masked(a, k, acc[a][0]);
    if (f_out.p[0] == nullptr) {
#pragma unroll
      for (int a = 0; a < 7; ++a)
        if (hasf<FM>(a)) du.p[a][o] = Fv[a];
      return;
    }
    T uin[7], fin[7];
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      uin[a] = T(0);
      fin[a] = T(0);
      if (hasf<FM>(a)) {
        uin[a] = (du_mode & DU_READ) ? du.p[a][o] : T(0);
        fin[a] = f.p[a][o];
      }
    }
#pragma unroll
    for (int a = 0; a < 7; ++a)
      if (hasf<FM>(a)) update(a, o, Fv[a], uin[a], fin[a]);
  };

  for (int r = it.z0 - 3; r <= it.z1 + 2; ++r) {
    const int kb = r - 3;
    const bool inch = r >= it.z0 && r < it.z1;
    if (valid(r)) {
      const int k = kk(r);
      const long long o = col(r);
      __syncthreads();
      if (inch) {
        const T* xs[8] = {f.p[1], ws.pq(POUT_GXX), ws.pq(POUT_GYX), ws.pq(POUT_LYZ),
                          ws.pq(POUT_HX), ws.q(QOUT_GZX), ws.q(QOUT_LZY), ws.q(QOUT_EY)};
        const T* ys[8] = {f.p[2], ws.pq(POUT_GXY), ws.pq(POUT_LXZ), ws.pq(POUT_GYY),
                          ws.pq(POUT_HY), ws.q(QOUT_GZY), ws.q(QOUT_LZX), ws.q(QOUT_EX)};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (hasf<FM>(kXOwn[q])) load_plane(sx + strip_slot<FM>(kXOwn, q) * PXs::NP, xs[q], b, ix, k);
          if (hasf<FM>(kYOwn[q])) load_plane(sy + strip_slot<FM>(kYOwn, q) * PYs::NP, ys[q], b, iy, k);
        }
        if (kQz) load_plane(s2, ws.pq(POUT_QZ), b, i3, k);
        if (kEz) load_plane(s2 + kQz * P3::NP, ws.pq(POUT_EZ), b, i3, k);
      }
      if (hasf<FM>(4)) {
        load_plane(sx + strip_slot<FM>(kXOwn, 8) * PXs::NP, ws.q(QOUT_QY), b, ix, k);
        load_plane(sy + strip_slot<FM>(kYOwn, 8) * PYs::NP, ws.q(QOUT_QX), b, iy, k);
      }
      if (kDB && kd != T(0)) {
        load_plane(sdb, ws.arr(WS_DIVB), b, ix, k);
        load_plane(sdb + PXs::NP, ws.arr(WS_DIVB), b, iy, k);
      }
      if constexpr (kCori) {
        load_plane(sxc, f.p[1], b, ix, k);
        load_plane(sxc + PXs::NP, f.p[3], b, ix, k);
        load_plane(syc, f.p[2], b, iy, k);
        load_plane(syc + PYs::NP, f.p[3], b, iy, k);
      }
      // Bz's dU and f at this plane, fetched with the planes
      T bz_u = T(0), bz_f = T(0);
      if (hasf<FM>(7) && inch && own && f_out.p[0] != nullptr) {
        if (du_mode & DU_READ) bz_u = du.p[7][o];
        bz_f = f.p[7][o];
      }
      __syncthreads();
      const int x = tx, y = ty;
      if (inch) {
        if (hasf<FM>(0) && cont)
          acc[0][3] += -(op6<1, 1, T>([&](int m) { return X(0, x + m); }, g.hxi) +
                         op6<1, 1, T>([&](int m) { return Y(0, y + m); }, g.hyi));
        if (hasf<FM>(1))
        acc[1][3] += op6<1, 0, T>([&](int m) { return X(1, x + m); }, g.hxi) +
                     op6<1, 1, T>([&](int m) { return Y(1, y + m); }, g.hyi) -
                     op6<0, 1, T>([&](int m) { return Y(2, y + m); }, T(0)) * inv_mu -
                     ws.pq(POUT_DPX)[o];
        if (hasf<FM>(2))
        acc[2][3] += op6<1, 0, T>([&](int m) { return Y(3, y + m); }, g.hyi) +
                     op6<1, 1, T>([&](int m) { return X(2, x + m); }, g.hxi) +
                     op6<0, 1, T>([&](int m) { return X(3, x + m); }, T(0)) * inv_mu -
                     ws.pq(POUT_DPY)[o];
        if (hasf<FM>(3)) {
          acc[3][3] -= ws.q(QOUT_DPZ)[o];
          acc[3][3] += op6<1, 1, T>([&](int m) { return X(5, x + m); }, g.hxi) +
                       op6<1, 1, T>([&](int m) { return Y(5, y + m); }, g.hyi) +
                       (op6<0, 1, T>([&](int m) { return Y(6, y + m); }, T(0)) -
                        op6<0, 1, T>([&](int m) { return X(6, x + m); }, T(0))) * inv_mu;
        }
        if (hasf<FM>(4))
        acc[4][3] += ws.pq(POUT_QC)[o] + ws.q(QOUT_CZZ)[o] +
                     op6<1, 1, T>([&](int m) { return X(4, x + m); }, g.hxi) +
                     op6<1, 1, T>([&](int m) { return Y(4, y + m); }, g.hyi) +
                     op6<0, 1, T>([&](int m) {
                       return op6<0, 1, T>([&](int a) { return F2(0, x + a, y + m); }, T(0));
                     }, T(0));
        // Newtonian cooling (eq. NewtonCool, eq. rhocool) at the cell centre
        if (hasf<FM>(4) && (tm & T_COOL)) {
          const T rc = f.p[0][o], ec = f.p[4][o];
          T q = -rc * (ec / rc - ph.e_cool) * ph.inv_tcool;
          if (ph.cool_cut) {
            const T r = rc * ph.inv_rho_cool, r2 = r * r;
            q = q * ((ph.cool_cut == 1 ? r2 : T(1)) / (T(1) + r2));
          }
          acc[4][3] += q;
        }
        if (hasf<FM>(5)) acc[5][3] += -op6<1, 1, T>([&](int m) { return F2(1, x, y + m); }, g.hyi);
        if (hasf<FM>(6)) acc[6][3] += op6<1, 1, T>([&](int m) { return F2(1, x + m, y); }, g.hxi);
        if (kDB && kd != T(0)) {
          acc[5][3] += kd * op6<1, 0, T>([&](int m) { return sdb[PXs::at(x + m, ty)]; }, g.hxi);
          acc[6][3] += kd * op6<1, 0, T>([&](int m) { return sdb[PXs::NP + PYs::at(tx, y + m)]; }, g.hyi);
        }
        // Bz has no z divergence: complete at once
        if (hasf<FM>(7) && own) {
          T fbz = -(op6<1, 1, T>([&](int m) { return X(7, x + m); }, g.hxi) -
                    op6<1, 1, T>([&](int m) { return Y(7, y + m); }, g.hyi));
          if (kd != T(0)) {
            // z part of grad(div B) on this z-face, from the own column
            const T* __restrict__ dbg = ws.arr(WS_DIVB);
            T w[6];
#pragma unroll
            for (int m = 0; m < 6; ++m) w[m] = valid(r - 3 + m) ? dbg[col(r - 3 + m)] : T(0);
            fbz += kd * zwin<1, 0, 6, 3>(w, r, wall, N, g.hzi, zt);
          }
          const T F7 = masked(7, r, fbz);
          if (f_out.p[0] == nullptr) du.p[7][o] = F7;
          else update(7, o, F7, bz_u, bz_f);
        }
      }
      // Coriolis force (eq. mom): -2 Omega x p, each component on its own
      // face; the parts that end with an interpolation along z, scattered
      // below (the in-plane parts arrive with pass P's face terms)
      T czx = T(0), czy = T(0), czz = T(0);
      if constexpr (kCori) {
        const T wx = ph.cor2[0], wy = ph.cor2[1];
        czx = -wy * op6<0, 0, T>([&](int m) { return XC(1, x + m); }, T(0));
        czy = wx * op6<0, 0, T>([&](int n) { return YC(1, y + n); }, T(0));
        czz = wy * op6<0, 1, T>([&](int m) { return XC(0, x + m); }, T(0)) -
              wx * op6<0, 1, T>([&](int n) { return YC(0, y + n); }, T(0));
      }
      T xqy = T(0), yqx = T(0);
      if (hasf<FM>(4)) {
        xqy = op6<0, 1, T>([&](int m) { return X(8, x + m); }, T(0));
        yqx = op6<0, 1, T>([&](int m) { return Y(8, y + m); }, T(0));
      }
      // ---- z divergences of plane r scattered into output planes r-3..r+3:
      // derivatives through first differences, interpolations directly
      T cur[7];
      const T* cols[7] = {f.p[3], ws.q(QOUT_GXZ), ws.q(QOUT_GYZ), ws.q(QOUT_GZZ), ws.q(QOUT_HZ),
                          ws.q(QOUT_EY), ws.q(QOUT_EX)};
#pragma unroll
      for (int a = 0; a < 7; ++a) cur[a] = hasf<FM>(a) ? cols[a][o] : T(0);
      T dl[7];
#pragma unroll
      for (int a = 0; a < 7; ++a) {
        dl[a] = (cur[a] - prev[a]) * g.hzi;
        prev[a] = cur[a];
      }
      if (hasf<FM>(0) && cont) zscatter_d<1, 3>(acc[0], kb, -dl[0], wall, N, zt);
      if (hasf<FM>(1)) {
        zscatter_d<1, 3>(acc[1], kb, dl[1], wall, N, zt);
        zscatter<0, 1, 3>(acc[1], kb, ws.q(QOUT_LXY)[o] * inv_mu, wall, N, zt);
        if constexpr (kCori) zscatter<0, 1, 3>(acc[1], kb, czx, wall, N, zt);
      }
      if (hasf<FM>(2)) {
        zscatter_d<1, 3>(acc[2], kb, dl[2], wall, N, zt);
        zscatter<0, 1, 3>(acc[2], kb, -ws.q(QOUT_LYX)[o] * inv_mu, wall, N, zt);
        if constexpr (kCori) zscatter<0, 1, 3>(acc[2], kb, czy, wall, N, zt);
      }
      if (hasf<FM>(3)) {
        zscatter_d<0, 3>(acc[3], kb, dl[3], wall, N, zt);
        if (grav) zscatter<0, 0, 3>(acc[3], kb, -f.p[0][o] * ph.gz, wall, N, zt);
        if constexpr (kCori) zscatter<0, 0, 3>(acc[3], kb, czz, wall, N, zt);
      }
      if (hasf<FM>(4)) {
        zscatter_d<1, 3>(acc[4], kb, dl[4], wall, N, zt);
        zscatter<0, 1, 3>(acc[4], kb, xqy, wall, N, zt);
        zscatter<0, 1, 3>(acc[4], kb, yqx, wall, N, zt);
      }
      if (hasf<FM>(5)) zscatter_d<1, 3>(acc[5], kb, dl[5], wall, N, zt);
      if (hasf<FM>(6)) zscatter_d<1, 3>(acc[6], kb, -dl[6], wall, N, zt);
    } else {
#pragma unroll
      for (int a = 0; a < 7; ++a) prev[a] = T(0);
    }
    // ---- plane kb = r-3 is complete
    if (own && valid(kb) && kb >= it.z0 && kb < it.z1) finalize7(kb);
#pragma unroll
    for (int a = 0; a < 7; ++a) {
#pragma unroll
      for (int s = 0; s < 6; ++s) acc[a][s] = acc[a][s + 1];
      acc[a][6] = T(0);
    }
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
  hipLaunchKernelGGL((zA1<T, TX, TY, false, true>), grid, block, 0, L.stream, L.boxes, L.items, n, ztab,
                     (int*)nullptr, f, ph, w, (CPart*)nullptr, dfdt, red);
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

// ---------------------------------------------------------------------------
template <class T, int TX, int TY, bool PERS, unsigned FM, class G>
static void zF_one(const G& grid, dim3 block, const ZLaunch& L, const ZStageArgs<T>& a, int* q) {
  hipLaunchKernelGGL((zF<T, TX, TY, PERS, FM>), grid((const void*)zF<T, TX, TY, PERS, FM>), block, 0, L.stream,
                     L.boxes, L.fitems, L.nfitems, a.ztab, q, a.f, a.w, a.ph, a.du, a.du_mode, a.f_out, a.alpha,
                     a.beta, a.dt_dev, a.dt_host);
}
// The momentum launch's mask with the Coriolis bit (8) set; others unchanged.
template <unsigned FM> constexpr unsigned with_cori() { return (FM & 0x0Eu) ? (FM | 0x100u) : FM; }
// one launch per mask, each with its own 8 queue counters
template <class T, int TX, int TY, bool PERS, class G, size_t... I>
static void zF_launch(const G& grid, dim3 block, const ZLaunch& L, const ZStageArgs<T>& a, int* q,
                      std::index_sequence<I...>) {
  if (a.ph.terms & T_CORI)
    (zF_one<T, TX, TY, PERS, with_cori<kFMasks[I]>()>(grid, block, L, a, q ? q + 32 + 8 * int(I) : q), ...);
  else
    (zF_one<T, TX, TY, PERS, kFMasks[I]>(grid, block, L, a, q ? q + 32 + 8 * int(I) : q), ...);
}

__global__ void k_qreset(int* q) {
  if ((int)threadIdx.x < kQueueInts) q[threadIdx.x] = 0;
}

// Workgroups of a kernel that fit on the device at once (cached per kernel).
static int resident_groups(const void* kern, int block, int ncu) {
  static std::mutex mu;
  static std::map<const void*, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(kern);
  if (it != cache.end()) return it->second;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, block, 0) != hipSuccess || nb < 1) nb = 1;
  return cache[kern] = nb * ncu;
}

// Pass F, in its own tile shape (L.ftile) over its own work items.
template <class T, int TX, int TY, bool PERS>
static void launch_final_t(const ZLaunch& L, const ZStageArgs<T>& a, int* q) {
  const int n = L.nfitems;
  auto grid = [&](const void* kern) {
    if (!q) return dim3(8 * ((n + 7) / 8));
    const int r = std::min(n, resident_groups(kern, TX * TY, L.ncu));
    return dim3(std::max(8, r - r % 8));
  };
  zF_launch<T, TX, TY, PERS>(grid, dim3(TX * TY), L, a, q, std::make_index_sequence<kNFMasks>{});
}

template <class T, bool PERS>
static void launch_final(const ZLaunch& L, const ZStageArgs<T>& a, int* q) {
  switch (L.ftile) {
    case ZTILE_32x8: launch_final_t<T, 32, 8, PERS>(L, a, q); break;
    case ZTILE_16x16: launch_final_t<T, 16, 16, PERS>(L, a, q); break;
    case ZTILE_16x8: launch_final_t<T, 16, 8, PERS>(L, a, q); break;
    case ZTILE_64x8: launch_final_t<T, 64, 8, PERS>(L, a, q); break;
    default: launch_final_t<T, 64, 4, PERS>(L, a, q); break;
  }
}

template <class T, int TX, int TY, bool PERS>
static void launch_zstage_m(const ZLaunch& L, const ZStageArgs<T>& a) {
  const int n = L.nitems;
  const dim3 block(TX * TY);
  int* q = PERS ? L.queue : nullptr;
  auto grid = [&](const void* kern) {
    if (!q) return dim3(8 * ((n + 7) / 8));
    const int r = std::min(n, resident_groups(kern, TX * TY, L.ncu));
    return dim3(std::max(8, r - r % 8));
  };
  if (q) hipLaunchKernelGGL(k_qreset, dim3(1), dim3(64), 0, L.stream, q);
  L.at(PASS_PRIM);
  hipLaunchKernelGGL((zA1<T, TX, TY, PERS>), grid((const void*)zA1<T, TX, TY, PERS>), block, 0, L.stream, L.boxes,
                     L.items, n, a.ztab, q, a.f, a.ph, a.w, a.cpart);
  L.at(PASS_MEAN3);
  hipLaunchKernelGGL((zA2<T, TX, TY, PERS>), grid((const void*)zA2<T, TX, TY, PERS>), block, 0, L.stream, L.boxes,
                     L.items, n, a.ztab, q ? q + 8 : q, a.w, a.cpart);
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
  hipLaunchKernelGGL((zQ<T, TX, TY, PERS, QM_EDGES>), grid((const void*)zQ<T, TX, TY, PERS, QM_EDGES>), block, 0,
                     L.stream, L.boxes, L.items, n, a.ztab, q ? q + 16 : q, a.f, a.ph, a.w, a.lnavg,
                     a.w.lnpav);
  if (lnp)
    hipLaunchKernelGGL((zQ<T, TX, TY, PERS, QM_ZC | QM_LNP>), grid((const void*)zQ<T, TX, TY, PERS, QM_ZC | QM_LNP>),
                       block, 0, L.stream, L.boxes, L.items, n, a.ztab, q ? q + 32 + 8 * kNFMasks : q, a.f, a.ph,
                       a.w, a.lnavg, a.w.lnpav);
  else
    hipLaunchKernelGGL((zQ<T, TX, TY, PERS, QM_ZC>), grid((const void*)zQ<T, TX, TY, PERS, QM_ZC>), block, 0,
                       L.stream, L.boxes, L.items, n, a.ztab, q ? q + 32 + 8 * kNFMasks : q, a.f, a.ph, a.w,
                       a.lnavg, a.w.lnpav);
  L.at(PASS_CF);
  hipLaunchKernelGGL((zP<T, TX, TY, PERS>), grid((const void*)zP<T, TX, TY, PERS>), block, 0, L.stream, L.boxes,
                     L.items, n, a.ztab, q ? q + 24 : q, a.f, a.ph, a.w);
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
    default:
      launch_zstage_t<T, 64, 4>(L, a);
      break;
  }
}

template void launch_zstage<float>(const ZLaunch&, const ZStageArgs<float>&);
template void launch_zstage<double>(const ZLaunch&, const ZStageArgs<double>&);

}  // namespace smhd
