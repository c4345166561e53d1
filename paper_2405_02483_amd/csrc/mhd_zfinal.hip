// Pass F of an RK stage: every divergence of the stage's edge, centre and
// face quantities and of the momenta, gravity, the wall masking and the
// fused RK stage update (eqs. mass, mom, ien, indu; eqs. ddt, tupdate).
//
// x/y divergences of plane r read LDS strips; z divergences are scattered
// into per-thread accumulators of output planes r-3..r+3 (first differences
// for derivatives), and plane r-3 is then complete.
//
// Pass P's in-plane quantities (z-edge, centre and x/y face terms;
// mhd_zstage.hpp) come from the stage workspace as strips; each launch
// completes one field group (kFMasks) and loads only that group's strips.
#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

#include "mhd_zmarch.hpp"
#include "mhd_zstage.hpp"

namespace smhd {

// the field each LDS strip serves, in F's strip order: x strips, y strips
constexpr int kXOwn[9] = {0, 1, 2, 2, 4, 3, 3, 7, 4};
constexpr int kYOwn[9] = {0, 1, 1, 2, 4, 3, 3, 7, 4};
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
                                              const ZItem* __restrict__ items, int nitems,
                                              const T* __restrict__ ztab, int* __restrict__ queue,
                                              CP8<T> f, ZWork<T> ws, Phys<T> ph, P8<T> du,
                                              int du_mode, P8<T> f_out, T alpha, double beta,
                                              const double* __restrict__ dt_dev, double dt_host) {
  using PXs = Plane<TX, TY, 3, 0>;   // x-halo strips
  using PYs = Plane<TX, TY, 0, 3>;   // y-halo strips
  using P3 = Plane<TX, TY, 3>;
  // x strips: 0 px 1 Gxx 2 Gyx 3 Lyz 4 Hx 5 Gzx 6 Lzy 7 Ey 8 Qy
  // y strips: 0 py 1 Gxy 2 Lxz 3 Gyy 4 Hy 5 Gzy 6 Lzx 7 Ex 8 Qx
  // full:     0 Qz 1 Ez
  constexpr bool kQz = hasf<FM>(4), kEz = hasf<FM>(5) || hasf<FM>(6);
  // Coriolis force (bit 8 of FM; its in-plane parts come with the face
  // pressure gradients): x strips of px and pz, y strips of py and pz
  constexpr bool kCori = hasf<FM>(8);
  // div B diffusion (with the B_x launch): x and y strips of div B
  constexpr bool kDB = hasf<FM>(5);
  // a stretched z axis (bit 9): z derivatives scattered with each output
  // plane's Jacobian
  constexpr bool kStr = hasf<FM>(9);
  // only the strips of this launch's fields occupy LDS
  __shared__ T sx[at_least1(strip_slot<FM>(kXOwn, 9)) * PXs::NP];
  __shared__ T sy[at_least1(strip_slot<FM>(kYOwn, 9)) * PYs::NP];
  __shared__ T s2[at_least1(int(kQz) + int(kEz)) * P3::NP];
  __shared__ T sxc[kCori ? 2 * PXs::NP : 1];
  __shared__ T syc[kCori ? 2 * PYs::NP : 1];
  __shared__ T sdb[kDB ? PXs::NP + PYs::NP : 1];
  ZLOOP_BEGIN
  PlaneIdx<TX, TY, 3, 0> ix;
  PlaneIdx<TX, TY, 0, 3> iy;
  ix.init(b, it.x0, it.y0);
  iy.init(b, it.x0, it.y0);
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
  auto XC = [&](int q, int x) -> T { return sxc[q * PXs::NP + PXs::at(x, ty)]; };   // 0 px 1 pz
  auto YC = [&](int q, int y) -> T { return syc[q * PYs::NP + PYs::at(tx, y)]; };   // 0 py 1 pz
  auto DBX = [&](int x) -> T { return sdb[PXs::at(x, ty)]; };
  auto DBY = [&](int y) -> T { return sdb[PXs::NP + PYs::at(tx, y)]; };

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

  PlaneIdx<TX, TY, 3> i3;
  i3.init(b, it.x0, it.y0);

  for (int r = it.z0 - 3; r <= it.z1 + 2; ++r) {
    const int kb = r - 3;
    const bool inch = r >= it.z0 && r < it.z1;
    if (valid(r)) {
      const int k = kk(r);
      const long long o = col(r);
      const int x = tx, y = ty;
      __syncthreads();
      // ---- loads of plane r
      const T* qxs[4] = {ws.q(QOUT_GZX), ws.q(QOUT_LZY), ws.q(QOUT_EY), ws.q(QOUT_QY)};
      const T* qys[4] = {ws.q(QOUT_GZY), ws.q(QOUT_LZX), ws.q(QOUT_EX), ws.q(QOUT_QX)};
      if (inch) {
        const T* xs[8] = {f.p[1], ws.pq(POUT_GXX), ws.pq(POUT_GYX), ws.pq(POUT_LYZ),
                          ws.pq(POUT_HX), qxs[0], qxs[1], qxs[2]};
        const T* ys[8] = {f.p[2], ws.pq(POUT_GXY), ws.pq(POUT_LXZ), ws.pq(POUT_GYY),
                          ws.pq(POUT_HY), qys[0], qys[1], qys[2]};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (hasf<FM>(kXOwn[q])) load_plane(sx + strip_slot<FM>(kXOwn, q) * PXs::NP, xs[q], b, ix, k);
          if (hasf<FM>(kYOwn[q])) load_plane(sy + strip_slot<FM>(kYOwn, q) * PYs::NP, ys[q], b, iy, k);
        }
        if (kQz) load_plane(s2, ws.pq(POUT_QZ), b, i3, k);
        if (kEz) load_plane(s2 + kQz * P3::NP, ws.pq(POUT_EZ), b, i3, k);
      }
      if (hasf<FM>(4)) {
        load_plane(sx + strip_slot<FM>(kXOwn, 8) * PXs::NP, qxs[3], b, ix, k);
        load_plane(sy + strip_slot<FM>(kYOwn, 8) * PYs::NP, qys[3], b, iy, k);
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
      // own-column values of plane r for the z divergences
      T cur[7];
      const T* cols[7] = {f.p[3], ws.q(QOUT_GXZ), ws.q(QOUT_GYZ), ws.q(QOUT_GZZ), ws.q(QOUT_HZ),
                          ws.q(QOUT_EY), ws.q(QOUT_EX)};
#pragma unroll
      for (int a = 0; a < 7; ++a) cur[a] = hasf<FM>(a) ? cols[a][o] : T(0);
      const T lxy = hasf<FM>(1) ? ws.q(QOUT_LXY)[o] : T(0);
      const T lyx = hasf<FM>(2) ? ws.q(QOUT_LYX)[o] : T(0);
      const T rho_o = (hasf<FM>(3) && grav) ? f.p[0][o] : T(0);
      // own-cell terms of the own planes
      T dpx = T(0), dpy = T(0), qc = T(0), dpz = T(0), czz_ = T(0);
      if (inch) {
        if (hasf<FM>(3)) dpz = ws.q(QOUT_DPZ)[o];
        if (hasf<FM>(4)) czz_ = ws.q(QOUT_CZZ)[o];
        if (hasf<FM>(1)) dpx = ws.pq(POUT_DPX)[o];
        if (hasf<FM>(2)) dpy = ws.pq(POUT_DPY)[o];
        if (hasf<FM>(4)) qc = ws.pq(POUT_QC)[o];
      }
      // Bz's dU and f at this plane, fetched with the planes
      T bz_u = T(0), bz_f = T(0);
      if (hasf<FM>(7) && inch && own && f_out.p[0] != nullptr) {
        if (du_mode & DU_READ) bz_u = du.p[7][o];
        bz_f = f.p[7][o];
      }
      __syncthreads();
      if (inch) {
        if (hasf<FM>(0) && cont)
          acc[0][3] += -(op6<1, 1, T>([&](int m) { return X(0, x + m); }, g.hxi) +
                         op6<1, 1, T>([&](int m) { return Y(0, y + m); }, g.hyi));
        if (hasf<FM>(1))
          acc[1][3] += op6<1, 0, T>([&](int m) { return X(1, x + m); }, g.hxi) +
                       op6<1, 1, T>([&](int m) { return Y(1, y + m); }, g.hyi) -
                       op6<0, 1, T>([&](int m) { return Y(2, y + m); }, T(0)) * inv_mu - dpx;
        if (hasf<FM>(2))
          acc[2][3] += op6<1, 0, T>([&](int m) { return Y(3, y + m); }, g.hyi) +
                       op6<1, 1, T>([&](int m) { return X(2, x + m); }, g.hxi) +
                       op6<0, 1, T>([&](int m) { return X(3, x + m); }, T(0)) * inv_mu - dpy;
        if (hasf<FM>(3)) {
          acc[3][3] -= dpz;
          acc[3][3] += op6<1, 1, T>([&](int m) { return X(5, x + m); }, g.hxi) +
                       op6<1, 1, T>([&](int m) { return Y(5, y + m); }, g.hyi) +
                       (op6<0, 1, T>([&](int m) { return Y(6, y + m); }, T(0)) -
                        op6<0, 1, T>([&](int m) { return X(6, x + m); }, T(0))) * inv_mu;
        }
        if (hasf<FM>(4))
          acc[4][3] += qc + czz_ +
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
            const T rr = rc * ph.inv_rho_cool, r2 = rr * rr;
            q = q * ((ph.cool_cut == 1 ? r2 : T(1)) / (T(1) + r2));
          }
          acc[4][3] += q;
        }
        if (hasf<FM>(5)) acc[5][3] += -op6<1, 1, T>([&](int m) { return F2(1, x, y + m); }, g.hyi);
        if (hasf<FM>(6)) acc[6][3] += op6<1, 1, T>([&](int m) { return F2(1, x + m, y); }, g.hxi);
        if (kDB && kd != T(0)) {
          acc[5][3] += kd * op6<1, 0, T>([&](int m) { return DBX(x + m); }, g.hxi);
          acc[6][3] += kd * op6<1, 0, T>([&](int m) { return DBY(y + m); }, g.hyi);
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
            fbz += kd * zwin<1, 0, 6, 3>(w, r, wall, N, zj(r, ZJ_F), zt);
          }
          const T F7 = masked(7, r, fbz);
          if (f_out.p[0] == nullptr) du.p[7][o] = F7;
          else update(7, o, F7, bz_u, bz_f);
        }
      }
      // Coriolis force (eq. mom): -2 Omega x p, each component on its own
      // face; the parts that end with an interpolation along z, scattered
      // below (the in-plane parts arrive with the face pressure gradients)
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
      T dl[7];
#pragma unroll
      for (int a = 0; a < 7; ++a) {
        dl[a] = kStr ? cur[a] - prev[a] : (cur[a] - prev[a]) * g.hzi;
        prev[a] = cur[a];
      }
      // Jacobians of the output planes kb..kb+6 (up: centres, dn: faces)
      T jsc[7], jsf[7];
      if constexpr (kStr) {
#pragma unroll
        for (int s = 0; s < 7; ++s) {
          jsc[s] = valid(kb + s) ? zj(kb + s, ZJ_C) : T(0);
          jsf[s] = valid(kb + s) ? zj(kb + s, ZJ_F) : T(0);
        }
      }
      auto scat_up = [&](T (&ac)[7], T dv) {
        if constexpr (kStr) zscatter_dj<1, 3>(ac, kb, dv, jsc, wall, N, zt);
        else zscatter_d<1, 3>(ac, kb, dv, wall, N, zt);
      };
      if (hasf<FM>(0) && cont) scat_up(acc[0], -dl[0]);
      if (hasf<FM>(1)) {
        scat_up(acc[1], dl[1]);
        zscatter<0, 1, 3>(acc[1], kb, lxy * inv_mu, wall, N, zt);
        if constexpr (kCori) zscatter<0, 1, 3>(acc[1], kb, czx, wall, N, zt);
      }
      if (hasf<FM>(2)) {
        scat_up(acc[2], dl[2]);
        zscatter<0, 1, 3>(acc[2], kb, -lyx * inv_mu, wall, N, zt);
        if constexpr (kCori) zscatter<0, 1, 3>(acc[2], kb, czy, wall, N, zt);
      }
      if (hasf<FM>(3)) {
        if constexpr (kStr) zscatter_dj<0, 3>(acc[3], kb, dl[3], jsf, wall, N, zt);
        else zscatter_d<0, 3>(acc[3], kb, dl[3], wall, N, zt);
        if (grav) zscatter<0, 0, 3>(acc[3], kb, -rho_o * ph.gz, wall, N, zt);
        if constexpr (kCori) zscatter<0, 0, 3>(acc[3], kb, czz, wall, N, zt);
      }
      if (hasf<FM>(4)) {
        scat_up(acc[4], dl[4]);
        zscatter<0, 1, 3>(acc[4], kb, xqy, wall, N, zt);
        zscatter<0, 1, 3>(acc[4], kb, yqx, wall, N, zt);
      }
      if (hasf<FM>(5)) scat_up(acc[5], dl[5]);
      if (hasf<FM>(6)) scat_up(acc[6], -dl[6]);
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

// ---------------------------------------------------------------------------
// Launchers.
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

int zresident_groups(const void* kern, int block, int ncu) { return resident_groups(kern, block, ncu); }

template <class T, int TX, int TY, bool PERS, unsigned FM, class G>
static void zF_one(const G& grid, dim3 block, const ZLaunch& L, const ZStageArgs<T>& a, int* q) {
  hipLaunchKernelGGL((zF<T, TX, TY, PERS, FM>), grid((const void*)zF<T, TX, TY, PERS, FM>), block, 0,
                     L.stream, L.boxes, L.fitems, L.nfitems, a.ztab, q, a.f, a.w, a.ph, a.du, a.du_mode, a.f_out,
                     a.alpha, a.beta, a.dt_dev, a.dt_host);
}
// The momentum launch's mask with the Coriolis bit (8) set; others unchanged.
template <unsigned FM> constexpr unsigned with_cori() { return (FM & 0x0Eu) ? (FM | 0x100u) : FM; }
// one launch per mask, each with its own 8 queue counters; a stretched z
// axis takes the instantiations with bit 9 (grid mode only)
template <class T, int TX, int TY, bool PERS, class G, size_t... I>
static void zF_launch(const G& grid, dim3 block, const ZLaunch& L, const ZStageArgs<T>& a, int* q,
                      std::index_sequence<I...>) {
  if constexpr (!PERS) {
    if (L.stretched) {
      if (a.ph.terms & T_CORI)
        (zF_one<T, TX, TY, false, with_cori<kFMasks[I]>() | 0x200u>(grid, block, L, a, nullptr), ...);
      else
        (zF_one<T, TX, TY, false, kFMasks[I] | 0x200u>(grid, block, L, a, nullptr), ...);
      return;
    }
  }
  if (a.ph.terms & T_CORI)
    (zF_one<T, TX, TY, PERS, with_cori<kFMasks[I]>()>(grid, block, L, a, q ? q + 32 + 8 * int(I) : q), ...);
  else
    (zF_one<T, TX, TY, PERS, kFMasks[I]>(grid, block, L, a, q ? q + 32 + 8 * int(I) : q), ...);
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
void launch_final(const ZLaunch& L, const ZStageArgs<T>& a, int* q) {
  if constexpr (PERS) {
    if (L.stretched) {   // the stretched instantiations run in grid mode
      launch_final<T, false>(L, a, nullptr);
      return;
    }
  }
  switch (L.ftile) {
    case ZTILE_32x8: launch_final_t<T, 32, 8, PERS>(L, a, q); break;
    case ZTILE_16x16: launch_final_t<T, 16, 16, PERS>(L, a, q); break;
    case ZTILE_16x8: launch_final_t<T, 16, 8, PERS>(L, a, q); break;
    case ZTILE_64x8: launch_final_t<T, 64, 8, PERS>(L, a, q); break;
    case ZTILE_32x16: launch_final_t<T, 32, 16, PERS>(L, a, q); break;
    default: launch_final_t<T, 64, 4, PERS>(L, a, q); break;
  }
}

template void launch_final<float, false>(const ZLaunch&, const ZStageArgs<float>&, int*);
template void launch_final<float, true>(const ZLaunch&, const ZStageArgs<float>&, int*);
template void launch_final<double, false>(const ZLaunch&, const ZStageArgs<double>&, int*);
template void launch_final<double, true>(const ZLaunch&, const ZStageArgs<double>&, int*);

}  // namespace smhd
