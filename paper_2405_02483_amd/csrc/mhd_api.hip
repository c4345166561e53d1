// C ABI of libstaggermhd (declared in include/mhd.h): context set-up,
// argument checks, workspace ownership and the sequencing of the kernel
// passes for mhd_rhs, mhd_step, mhd_step_adjoint, mhd_rhs_adjoint,
// mhd_reductions and mhd_divb_clean; the spline intervals of a stretched z
// axis and the per-plane and wall tables; the autotuner.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mhd.h"
#include "mhd_adjoint.hpp"
#include "mhd_clean.hpp"
#include "mhd_kernels.hpp"
#include "mhd_zmarch_api.hpp"

using namespace smhd;

struct mhd_ctx {
  mhd_params p;
  std::vector<mhd_box> boxes;
  std::vector<long long> offsets;
  long long nelem = 0;
  size_t esize = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  // device tables
  BoxDev* d_boxes = nullptr;
  Blk* d_tab = nullptr;
  int nblk = 0;
  Blk* d_gtab = nullptr;
  int ngblk = 0;
  std::vector<BoxDev> h_boxes;
  // workspace
  void* work = nullptr;            // work_arrays(p) * nelem elements
  RedItem* d_red = nullptr;        // per-item partials of mhd_reductions (nitems)
  RedTotal* d_tot = nullptr;       // their fold
  void* adj = nullptr;             // adjoint workspace (allocated on first use)
  size_t adj_bytes = 0;
  VPlan* prog = nullptr;           // the right-hand side as a program (adjoint)
  double prog_dt = 0.0;            // the dt it was built for (div B diffusion; 0: without)
  double* d_pm = nullptr;          // plane means of the program (V_PMEAN), per plane
  VFused* d_fused = nullptr;       // prog->fused in device memory
  VStep* d_bsteps = nullptr;       // prog->bsteps in device memory
  // z-march stage kernels: work items, tile shape, Courant partials, dt
  ZItem* d_items = nullptr;
  int nitems = 0;
  ZItem* d_fitems = nullptr;       // pass F's own work items (tile ftile)
  int nfitems = 0;
  int ftile = ZTILE_32x8;
  int tile = ZTILE_32x8;
  CPart* d_cpart = nullptr;
  int* d_queue = nullptr;          // item queues of the persistent launch mode
  int persistent = 0;
  int ncu = 1;
  double* d_dt = nullptr;
  void* d_ztab = nullptr;          // z-coefficient tables of wall boxes (ctx dtype)
  void* d_lnavg = nullptr;         // ln of the plane means of e_m, per plane of every box
  double* d_lnpart = nullptr;      // their partial sums, kPlaneSlices per plane
  void* d_lnpav = nullptr;         // ln of the plane means of P, per plane of every box
  int nplanes = 0;
  void* scratch = nullptr;         // this device's address of the static scratch array
  CleanState* clean = nullptr;     // div B cleaning: rocFFT plans and scratch (first use)
  // stretched z axes: per box the grid intervals at the centres and faces
  // (empty for a uniform box)
  std::vector<std::vector<double>> dzc, dzf;
  int stretched = 0;
  // timing of kernel passes (mhd_profile)
  bool prof = false;
  std::vector<std::pair<int, hipEvent_t>> marks;
  double prof_ms[PASS_COUNT] = {};
  long long prof_n[PASS_COUNT] = {};
};

static void prof_mark(void* vc, int pass) {
  mhd_ctx* c = static_cast<mhd_ctx*>(vc);
  hipEvent_t ev;
  if (hipEventCreate(&ev) != hipSuccess) return;
  (void)hipEventRecord(ev, c->stream);
  c->marks.emplace_back(pass, ev);
}

// Fold recorded marks into per-pass totals (waits for the stream).
static int prof_fold(mhd_ctx* c) {
  if (c->marks.empty()) return MHD_OK;
  hipError_t e = hipStreamSynchronize(c->stream);
  for (size_t q = 0; q + 1 < c->marks.size(); ++q) {
    const int pass = c->marks[q].first;
    if (pass < 0 || pass >= PASS_COUNT) continue;
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->marks[q].second, c->marks[q + 1].second);
    c->prof_ms[pass] += ms;
    c->prof_n[pass] += 1;
  }
  for (auto& m : c->marks) (void)hipEventDestroy(m.second);
  c->marks.clear();
  return e == hipSuccess ? MHD_OK : MHD_EHIP;
}

static std::string g_init_err;

// The static scratch of mhd_rhs_noalloc (mhd.h): the stage workspace, the
// per-plane tables and the queue counters of one call, for callers that
// cannot allocate.  Each device that loads the library holds its own copy
// until the process ends.  Host code never uses this name as an address:
// scratch_address() gives each device's copy through hipGetSymbolAddress.
static constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// This device's address of `scratch` (the device must be current),
// resolved once per device.
static hipError_t scratch_address(int dev, void** out) {
  static std::mutex mu;
  static std::vector<void*> addr;
  std::lock_guard<std::mutex> lock(mu);
  if (dev < 0) return hipErrorInvalidDevice;
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

static const double kAlpha[3] = {0.0, -0.641874, -1.31021};   // eq. tconst
static const double kBeta[3] = {0.46173, 0.924087, 0.390614};

// Left end s of the real interval [-s, 0] on which one step of the
// low-storage RK3 scheme (eqs. ddt, tupdate, tconst, coefficients as printed)
// does not amplify y' = lambda y, z = lambda dt: |R(z)| <= 1 (about 2.5127).
static double rk3_real_limit() {
  auto amp = [](double z) {
    double f = 1.0, U = 0.0;
    for (int s = 0; s < 3; ++s) {
      U = kAlpha[s] * U + z * f;
      f += kBeta[s] * U;
    }
    return std::fabs(f);
  };
  double s = 0.0;
  while (amp(-(s + 1e-3)) <= 1.0) s += 1e-3;
  double lo = s, hi = s + 1e-3;
  for (int it = 0; it < 60; ++it) {
    const double m = 0.5 * (lo + hi);
    (amp(-m) <= 1.0 ? lo : hi) = m;
  }
  return lo;
}

// Largest stable c_divb of a box: the div B diffusion c h_min^2 / dt
// grad(div B) has eigenvalues -c h_min^2 / dt sum_a K_a^2 on longitudinal
// modes, K_a the symbol of the staggered derivative, largest at the
// two-cell wave: K_a h_a = 2 (75/64 + 25/384 + 3/640).  Stability of the RK3
// step needs c h_min^2 K^2 sum_a 1/h_a^2 <= rk3_real_limit(); on cubic cells
// c <= 0.1358.
static double divb_limit(double dx, double dy, double dz) {
  const double kh = 2.0 * (75.0 / 64.0 + 25.0 / 384.0 + 3.0 / 640.0);
  const double h = std::min(dx, std::min(dy, dz));
  const double s = h * h * (1.0 / (dx * dx) + 1.0 / (dy * dy) + 1.0 / (dz * dz));
  return rk3_real_limit() / (kh * kh * s);
}
// Stage workspace arrays: 34, 6 more for the quenched stress, and 2 more
// for the second-order switch.
static int work_arrays(const mhd_params& p) {
  if (p.terms & MHD_T_ORDER2) return WS_COUNT_ALL;
  return (p.terms & MHD_T_QUENCH) ? WS_COUNT_QUENCH : WS_COUNT;
}

// Grid intervals dz/dxi of a stretched z axis (Section 4.2: the Jacobian is
// the inverse of the spline-fitted grid interval at the derivative's
// centre): the not-a-knot cubic spline through (k, z[k]), k = 0..n-1, has
// second derivatives M with M[k-1] + 4 M[k] + M[k+1] = 6 (z[k+1] - 2 z[k] +
// z[k-1]) inside and M[0] - 2 M[1] + M[2] = 0, M[n-3] - 2 M[n-2] + M[n-1] =
// 0.  Subtracting the end rows from their neighbours gives M[1] and M[n-2]
// directly; rows 2..n-3 are tridiagonal in M[2..n-3].  Returns its
// derivative at the centres k (dzc) and the faces k - 1/2 (dzf; face 0 from
// the first interval's cubic).
static void zintervals(const std::vector<double>& z, std::vector<double>& dzc, std::vector<double>& dzf) {
  const int n = (int)z.size();
  std::vector<double> r(n, 0.0), M(n, 0.0);
  for (int k = 1; k < n - 1; ++k) r[k] = 6.0 * (z[k + 1] - 2.0 * z[k] + z[k - 1]);
  M[1] = r[1] / 6.0;
  M[n - 2] = r[n - 2] / 6.0;
  if (n > 4) {
    // Thomas algorithm on rows k = 2..n-3: M[k-1] + 4 M[k] + M[k+1] = r[k]
    const int a = 2, e = n - 3, m = e - a + 1;
    std::vector<double> cp(m), dp(m);
    for (int i = 0; i < m; ++i) {
      const int k = a + i;
      double rhs = r[k];
      if (k - 1 == 1) rhs -= M[1];
      if (k + 1 == n - 2) rhs -= M[n - 2];
      const double lo = i > 0 ? 1.0 : 0.0, up = i < m - 1 ? 1.0 : 0.0;
      const double den = 4.0 - lo * (i > 0 ? cp[i - 1] : 0.0);
      cp[i] = up / den;
      dp[i] = (rhs - lo * (i > 0 ? dp[i - 1] : 0.0)) / den;
    }
    for (int i = m - 1; i >= 0; --i) M[a + i] = dp[i] - (i < m - 1 ? cp[i] * M[a + i + 1] : 0.0);
  }
  M[0] = 2.0 * M[1] - M[2];
  M[n - 1] = 2.0 * M[n - 2] - M[n - 3];
  auto slope = [&](int k, double t) {   // S'(k + t) on [k, k+1]
    return -M[k] * (1.0 - t) * (1.0 - t) / 2.0 + M[k + 1] * t * t / 2.0 + (z[k + 1] - M[k + 1] / 6.0) -
           (z[k] - M[k] / 6.0);
  };
  dzc.resize(n);
  dzf.resize(n);
  for (int k = 0; k < n; ++k) {
    dzc[k] = k < n - 1 ? slope(k, 0.0) : slope(n - 2, 1.0);
    dzf[k] = k > 0 ? slope(k - 1, 0.5) : slope(0, -0.5);
  }
}

static int fail(mhd_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg; else g_init_err = msg;
  return code;
}

static int hipfail(mhd_ctx* c, hipError_t e, const char* what) {
  return fail(c, MHD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T> static Phys<T> make_phys(const mhd_params& p) {
  Phys<T> ph;
  ph.gamma = T(p.gamma);
  ph.gamma1 = T(p.gamma - 1.0);
  ph.mu = T(p.mu);
  ph.inv_mu = T(1.0 / p.mu);
  ph.gz = T(p.gz);
  ph.nu1 = T(p.nu1);
  ph.nu2 = T(p.nu2);
  ph.nu3 = T(p.nu3);
  ph.nu_const = T(p.nu_const);
  ph.c1 = T(p.c1);
  ph.nuE = T(p.nuE);
  ph.nuB = T(p.nuB);
  ph.eta_const = T(p.eta_const);
  const bool cool = p.terms & MHD_T_COOL;
  ph.e_cool = cool ? T(p.e_cool) : T(0);
  ph.inv_tcool = cool ? T(1.0 / p.t_cool) : T(0);
  ph.inv_rho_cool = cool && p.cool_cut ? T(1.0 / p.rho_cool) : T(0);
  ph.cool_cut = cool ? p.cool_cut : 0;
  const bool cori = p.terms & MHD_T_CORI;
  for (int a = 0; a < 3; ++a) ph.cor2[a] = cori ? T(2.0 * p.omega[a]) : T(0);
  ph.c_divb = (p.terms & MHD_T_DIVB) ? T(p.c_divb) : T(0);
  ph.c_smag = (p.terms & MHD_T_SMAG) ? T(p.c_smag) : T(0);
  const bool quench = p.terms & MHD_T_QUENCH;
  ph.q_max = quench ? T(p.q_max) : T(1);
  ph.q_lim = quench ? T(p.q_lim) : T(0);
  ph.d2_lim = (p.terms & MHD_T_ORDER2) ? T(p.d2_lim) : T(0);
  ph.terms = p.terms;
  return ph;
}

static Launch make_launch(const mhd_ctx* c) {
  Launch L;
  L.boxes = c->d_boxes;
  L.tab = c->d_tab;
  L.nblk = c->nblk;
  L.gtab = c->d_gtab;
  L.nghost_blk = c->ngblk;
  L.stream = c->stream;
  L.mark = c->prof ? prof_mark : nullptr;
  L.mark_ctx = const_cast<mhd_ctx*>(c);
  return L;
}

// Per-call device scratch of the stage kernels: the stage workspace, the
// per-plane tables and the persistent mode's queue counters.  Normally the
// context's own allocations; mhd_rhs_noalloc places them in the static
// array `scratch` instead.
struct Scratch {
  void* work;
  void* lnavg;
  void* lnpav;
  double* lnpart;
  int* queue;
};

static Scratch own_scratch(const mhd_ctx* c) {
  return Scratch{c->work, c->d_lnavg, c->d_lnpav, c->d_lnpart, c->d_queue};
}

template <class T> static ZWork<T> make_zwork(const mhd_ctx* c, const Scratch& s) {
  ZWork<T> w;
  w.base = static_cast<T*>(s.work);
  w.stride = c->nelem;
  w.lnpav = static_cast<T*>(s.lnpav);
  return w;
}
template <class T> static ZWork<T> make_zwork(const mhd_ctx* c) { return make_zwork<T>(c, own_scratch(c)); }

static ZLaunch make_zlaunch(const mhd_ctx* c, const Scratch& s) {
  ZLaunch L;
  L.boxes = c->d_boxes;
  L.items = c->d_items;
  L.nitems = c->nitems;
  L.tile = c->tile;
  L.fitems = c->d_fitems;
  L.nfitems = c->nfitems;
  L.ftile = c->ftile;
  L.queue = s.queue;
  L.persistent = c->persistent;
  L.ncu = c->ncu;
  L.nbox = (int)c->h_boxes.size();
  L.nplanes = c->nplanes;
  L.stretched = c->stretched;
  L.stream = c->stream;
  L.mark = c->prof ? prof_mark : nullptr;
  L.mark_ctx = const_cast<mhd_ctx*>(c);
  return L;
}
static ZLaunch make_zlaunch(const mhd_ctx* c) { return make_zlaunch(c, own_scratch(c)); }

// Work items of the z-march kernels: tiles of TX x TY columns, z split into
// chunks of about kZChunk planes (each chunk recomputes a few planes of
// lead-in).
#ifndef MHD_ZCHUNK
#define MHD_ZCHUNK 128
#endif
static constexpr int kZChunk = MHD_ZCHUNK;
// The z-range of an item: kZChunk planes, halved (down to kZChunkMin) while
// the items would number fewer than kItemsPerCU per compute unit, so that
// small boxes still fill the device.  The chunking changes no result: every
// output plane sums its z contributions in the same order.
static constexpr int kZChunkMin = 16, kItemsPerCU = 4;
static void build_items(const mhd_ctx* c, int tile, std::vector<ZItem>& items) {
  const int TX = ztile_x(tile), TY = ztile_y(tile);
  auto nchunks = [](int nzt, int chunk) { return std::max(1, (nzt + chunk / 2) / chunk); };
  int chunk = kZChunk;
  for (;;) {
    long long n = 0;
    for (const BoxDev& d : c->h_boxes)
      n += (long long)nchunks(d.nzt, chunk) * ((d.ny + TY - 1) / TY) * ((d.nx + TX - 1) / TX);
    if (n >= (long long)kItemsPerCU * c->ncu || chunk / 2 < kZChunkMin) break;
    chunk /= 2;
  }
  items.clear();
  for (int b = 0; b < (int)c->h_boxes.size(); ++b) {
    const BoxDev& d = c->h_boxes[b];
    const int nch = nchunks(d.nzt, chunk);
    for (int ch = 0; ch < nch; ++ch) {
      const int z0 = (int)((long long)d.nzt * ch / nch), z1 = (int)((long long)d.nzt * (ch + 1) / nch);
      for (int ty = 0; ty < d.ny; ty += TY)
        for (int tx = 0; tx < d.nx; tx += TX) {
          ZItem it;
          it.box = b;
          it.x0 = tx;
          it.y0 = ty;
          it.z0 = z0;
          it.z1 = z1;
          it.pad = 0;
          items.push_back(it);
        }
    }
  }
}

// Uploads the work items of a tile shape; *d and *n are replaced.  With
// cpart (the items of every pass but F), also the per-item Courant and
// reduction partials.
static int upload_items(mhd_ctx* c, int tile, ZItem** d, int* n, CPart** cpart) {
  std::vector<ZItem> items;
  build_items(c, tile, items);
  ZItem* di = nullptr;
  CPart* dp = nullptr;
  RedItem* dr = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&di, sizeof(ZItem) * items.size())) != hipSuccess ||
      (cpart && (e = hipMalloc(&dp, sizeof(CPart) * items.size())) != hipSuccess) ||
      (cpart && (e = hipMalloc(&dr, sizeof(RedItem) * items.size())) != hipSuccess)) {
    (void)hipFree(di);
    (void)hipFree(dp);
    return fail(c, MHD_ENOMEM, std::string("work item tables: ") + hipGetErrorString(e));
  }
  if ((e = hipMemcpy(di, items.data(), sizeof(ZItem) * items.size(), hipMemcpyHostToDevice)) != hipSuccess) {
    (void)hipFree(di);
    (void)hipFree(dp);
    (void)hipFree(dr);
    return hipfail(c, e, "work item upload");
  }
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  (void)hipFree(*d);
  *d = di;
  *n = (int)items.size();
  if (cpart) {
    (void)hipFree(*cpart);
    *cpart = dp;
    (void)hipFree(c->d_red);
    c->d_red = dr;
  }
  return MHD_OK;
}

// Pass F alone (its kernels read no per-item partials).
static int set_ftile(mhd_ctx* c, int tile) {
  const int rc = upload_items(c, tile, &c->d_fitems, &c->nfitems, nullptr);
  if (rc == MHD_OK) c->ftile = tile;
  return rc;
}

// Every pass.
static int set_tile(mhd_ctx* c, int tile) {
  int rc = upload_items(c, tile, &c->d_items, &c->nitems, &c->d_cpart);
  if (rc != MHD_OK) return rc;
  c->tile = tile;
  return set_ftile(c, tile);
}

template <class T> static P8<T> p8(void* const f[8]) {
  P8<T> r;
  for (int q = 0; q < 8; ++q) r.p[q] = static_cast<T*>(f[q]);
  return r;
}
template <class T> static CP8<T> cp8(void* const f[8]) {
  CP8<T> r;
  for (int q = 0; q < 8; ++q) r.p[q] = static_cast<const T*>(f ? f[q] : nullptr);
  return r;
}
template <class T> static CP8<T> cp8(const P8<T>& f) {
  CP8<T> r;
  for (int q = 0; q < 8; ++q) r.p[q] = f.p[q];
  return r;
}
template <class T> static P8<T> p8null() {
  P8<T> r;
  for (int q = 0; q < 8; ++q) r.p[q] = nullptr;
  return r;
}

static int check8(mhd_ctx* c, void* const f[8], const char* name) {
  if (!f) return fail(c, MHD_EINVAL, std::string(name) + " is NULL");
  for (int q = 0; q < 8; ++q) {
    if (!f[q]) return fail(c, MHD_EINVAL, std::string(name) + "[" + std::to_string(q) + "] is NULL");
    if (reinterpret_cast<uintptr_t>(f[q]) % 16 != 0)
      return fail(c, MHD_EINVAL, std::string(name) + " pointer not 16-byte aligned");
  }
  return MHD_OK;
}

static int check_launch(mhd_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hipfail(c, e, what);
  return MHD_OK;
}

// Block table: kBlock consecutive cells of one box per entry.
static void build_tables(mhd_ctx* c, std::vector<Blk>& tab, std::vector<Blk>& gtab) {
  for (int b = 0; b < (int)c->boxes.size(); ++b) {
    const BoxDev& d = c->h_boxes[b];
    for (long long s = 0; s < d.ncell; s += kBlock) {
      Blk t;
      t.box = b;
      t.start = s;
      t.n = (int)std::min<long long>(kBlock, d.ncell - s);
      tab.push_back(t);
    }
    if (d.wall) {
      const long long ng = (long long)d.nx * d.ny * 2 * d.ngz;
      for (long long s = 0; s < ng; s += kBlock) {
        Blk t;
        t.box = b;
        t.start = s;
        t.n = (int)std::min<long long>(kBlock, ng - s);
        gtab.push_back(t);
      }
    }
  }
}

extern "C" {

const char* mhd_last_error(const mhd_ctx* c) { return c ? c->err.c_str() : g_init_err.c_str(); }

int64_t mhd_field_elems(const mhd_ctx* c) { return c ? c->nelem : -1; }

int64_t mhd_box_offset(const mhd_ctx* c, int32_t b) {
  if (!c || b < 0 || b >= (int)c->offsets.size()) return -1;
  return c->offsets[b];
}

void mhd_destroy(mhd_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  for (auto& m : c->marks) (void)hipEventDestroy(m.second);
  (void)hipFree(c->d_boxes);
  (void)hipFree(c->d_tab);
  (void)hipFree(c->d_gtab);
  (void)hipFree(c->work);
  (void)hipFree(c->d_red);
  (void)hipFree(c->d_tot);
  (void)hipFree(c->adj);
  delete c->prog;
  (void)hipFree(c->d_pm);
  (void)hipFree(c->d_fused);
  (void)hipFree(c->d_bsteps);
  (void)hipFree(c->d_items);
  (void)hipFree(c->d_fitems);
  (void)hipFree(c->d_cpart);
  (void)hipFree(c->d_dt);
  (void)hipFree(c->d_queue);
  (void)hipFree(c->d_ztab);
  (void)hipFree(c->d_lnavg);
  (void)hipFree(c->d_lnpart);
  (void)hipFree(c->d_lnpav);
  clean_free(c->clean);
  delete c;
}

int mhd_init(const mhd_params* p, void* hip_stream, mhd_ctx** out) {
  if (!out) return fail(nullptr, MHD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p) return fail(nullptr, MHD_EINVAL, "params is NULL");
  if (p->dtype != MHD_F32 && p->dtype != MHD_F64) return fail(nullptr, MHD_EDTYPE, "unknown dtype");
  if (p->nbox < 1 || !p->boxes) return fail(nullptr, MHD_EINVAL, "need nbox >= 1 and a box array");
  if (!(p->gamma > 1.0) || !(p->mu > 0.0)) return fail(nullptr, MHD_EINVAL, "need gamma > 1 and mu > 0");
  const double nn[] = {p->nu1, p->nu2, p->nu3, p->nu_const, p->nuE, p->nuB, p->eta_const,
                       p->Cdt, p->Cdtd, p->Cdtr};
  for (double v : nn)
    if (!(v >= 0.0) || !std::isfinite(v)) return fail(nullptr, MHD_EINVAL, "viscosity, diffusion and Courant coefficients must be finite and >= 0");
  if (!std::isfinite(p->gz) || !std::isfinite(p->c1)) return fail(nullptr, MHD_EINVAL, "gz and c1 must be finite");
  if (p->terms & ~(MHD_T_ALL | MHD_T_COOL | MHD_T_CORI | MHD_T_EDIFFAV | MHD_T_LNP | MHD_T_DIVB |
                   MHD_T_SMAG | MHD_T_MAX5 | MHD_T_QUENCH | MHD_T_ORDER2))
    return fail(nullptr, MHD_EINVAL, "unknown term bits");
  if ((p->terms & MHD_T_DIVB) && !(p->c_divb >= 0.0 && std::isfinite(p->c_divb)))
    return fail(nullptr, MHD_EINVAL, "c_divb must be finite and >= 0");
  if ((p->terms & MHD_T_SMAG) && !(p->c_smag >= 0.0 && std::isfinite(p->c_smag)))
    return fail(nullptr, MHD_EINVAL, "c_smag must be finite and >= 0");
  if ((p->terms & MHD_T_QUENCH) && !(p->q_max > 0.0 && std::isfinite(p->q_max) && p->q_lim > 0.0 &&
                                     std::isfinite(p->q_lim)))
    return fail(nullptr, MHD_EINVAL, "q_max and q_lim must be finite and > 0");
  if ((p->terms & MHD_T_ORDER2) && !std::isfinite(p->d2_lim))
    return fail(nullptr, MHD_EINVAL, "d2_lim must be finite");
  if ((p->terms & MHD_T_CORI) &&
      !(std::isfinite(p->omega[0]) && std::isfinite(p->omega[1]) && std::isfinite(p->omega[2])))
    return fail(nullptr, MHD_EINVAL, "the rotation vector must be finite");
  if (p->reserved != 0 || p->reserved2 != 0) return fail(nullptr, MHD_EINVAL, "reserved fields must be 0");
  if (p->terms & MHD_T_COOL) {
    if (!std::isfinite(p->e_cool) || !(p->t_cool > 0.0) || !std::isfinite(p->t_cool))
      return fail(nullptr, MHD_EINVAL, "cooling needs a finite e_cool and a finite t_cool > 0");
    if (p->cool_cut < 0 || p->cool_cut > 2) return fail(nullptr, MHD_EINVAL, "cool_cut must be 0, 1 or 2");
    if (p->cool_cut != 0 && (!(p->rho_cool > 0.0) || !std::isfinite(p->rho_cool)))
      return fail(nullptr, MHD_EINVAL, "a cooling cut-off needs a finite rho_cool > 0");
  }

  mhd_ctx* c = new (std::nothrow) mhd_ctx();
  if (!c) return fail(nullptr, MHD_ENOMEM, "host allocation failed");
  c->p = *p;
  c->p.boxes = nullptr;
  c->esize = p->dtype == MHD_F32 ? sizeof(float) : sizeof(double);
  c->stream = static_cast<hipStream_t>(hip_stream);
  (void)hipGetDevice(&c->device);
  // the static scratch of mhd_rhs_noalloc; without it that call reports the
  // error and every other call works as usual
  if (scratch_address(c->device, &c->scratch) != hipSuccess) c->scratch = nullptr;
  if (hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
      c->ncu < 1)
    c->ncu = 1;
  long long off = 0;
  for (int b = 0; b < p->nbox; ++b) {
    const mhd_box& x = p->boxes[b];
    std::string where = "box " + std::to_string(b) + ": ";
    if (x.nx < 6 || x.ny < 6 || x.nz < 6) { delete c; return fail(nullptr, MHD_EINVAL, where + "need nx, ny, nz >= 6"); }
    if (x.reserved != 0) { delete c; return fail(nullptr, MHD_EINVAL, where + "reserved must be 0"); }
    if (x.bc_z == MHD_BC_PERIODIC) {
      if (x.ngz != 0) { delete c; return fail(nullptr, MHD_EINVAL, where + "periodic z needs ngz = 0"); }
    } else if (x.bc_z == MHD_BC_WALL) {
      if (x.ngz < 5) { delete c; return fail(nullptr, MHD_EINVAL, where + "walls need ngz >= 5"); }
      if (x.nz < x.ngz) { delete c; return fail(nullptr, MHD_EINVAL, where + "walls need nz >= ngz"); }
    } else {
      delete c;
      return fail(nullptr, MHD_EINVAL, where + "unknown bc_z");
    }
    if (!(x.Lx > 0) || !(x.Ly > 0) || !(x.Lz > 0)) { delete c; return fail(nullptr, MHD_EINVAL, where + "box sizes must be > 0"); }
    // a stretched z axis: the heights, copied, and their spline intervals
    std::vector<double> dzc, dzf;
    double dzmin = x.Lz / x.nz, dzmax = dzmin;
    if (x.zc) {
      if (x.bc_z != MHD_BC_WALL) { delete c; return fail(nullptr, MHD_EINVAL, where + "a stretched z axis needs walls"); }
      const int nzt = x.nz + 2 * x.ngz;
      std::vector<double> z(x.zc, x.zc + nzt);
      for (int k = 0; k < nzt; ++k)
        if (!std::isfinite(z[k]) || (k > 0 && !(z[k] > z[k - 1]))) {
          delete c;
          return fail(nullptr, MHD_EINVAL, where + "zc must be finite and strictly increasing");
        }
      zintervals(z, dzc, dzf);
      for (int k = 0; k < nzt; ++k)
        if (!(dzc[k] > 0.0) || !(dzf[k] > 0.0)) {
          delete c;
          return fail(nullptr, MHD_EINVAL, where + "the spline of zc is not increasing everywhere");
        }
      dzmin = *std::min_element(dzc.begin(), dzc.end());
      dzmax = *std::max_element(dzc.begin(), dzc.end());
      c->stretched = 1;
    }
    c->dzc.push_back(dzc);
    c->dzf.push_back(dzf);
    if ((p->terms & MHD_T_DIVB) && p->c_divb > divb_limit(x.Lx / x.nx, x.Ly / x.ny, dzmin)) {
      delete c;
      return fail(nullptr, MHD_EINVAL, where + "c_divb above the RK3 stability limit " +
                                           std::to_string(divb_limit(x.Lx / x.nx, x.Ly / x.ny, dzmin)));
    }
    if ((long long)x.nx * x.ny * (x.nz + 2LL * x.ngz) >= (1LL << 31)) {
      delete c;
      return fail(nullptr, MHD_EINVAL, where + "more than 2^31 - 1 cells (ghost planes included)");
    }
    c->boxes.push_back(x);
    c->boxes.back().zc = nullptr;    // the caller's array is not kept
    BoxDev d;
    d.nx = x.nx;
    d.ny = x.ny;
    d.nzt = x.nz + 2 * x.ngz;
    d.ngz = x.ngz;
    d.wall = x.bc_z == MHD_BC_WALL;
    d.g0 = x.ngz;
    d.g1 = x.ngz + x.nz;
    d.poff = c->nplanes;
    c->nplanes += d.nzt;
    d.off = off;
    d.ncell = (long long)d.nx * d.ny * d.nzt;
    d.dx = x.Lx / x.nx;
    d.dy = x.Ly / x.ny;
    d.dz = x.Lz / x.nz;
    d.hmin = std::min(d.dx, std::min(d.dy, dzmin));
    d.hmax = std::max(d.dx, std::max(d.dy, dzmax));
    d.stretched = x.zc ? 1 : 0;
    d.joff = -1;
    if (p->nu_const > 0.0) {
      for (int a = 0; a < 3; ++a) d.lv[a] = d.le[a] = d.hmin;
    } else {
      d.lv[0] = d.dx;
      d.lv[1] = d.dy;
      d.lv[2] = d.dz;
      d.le[0] = std::max(d.dx, d.dy);
      d.le[1] = std::max(d.dx, d.dz);
      d.le[2] = std::max(d.dy, d.dz);
    }
    d.zoff = -1;
    c->h_boxes.push_back(d);
    c->offsets.push_back(off);
    off += d.ncell;
  }
  c->nelem = off;
  // z-coefficient tables of the wall boxes
  std::vector<double> ztab;
  for (auto& d : c->h_boxes) {
    if (!d.wall) continue;
    d.zoff = (long long)ztab.size();
    for (int t = 0; t < ZT_COUNT; ++t)
      for (int k = 0; k < d.nzt; ++k)
        for (int dd = -3; dd <= 3; ++dd) {
          const int p = k + dd;
          ztab.push_back(p >= 0 && p < d.nzt ? zwall_coef(t, k, p, d.nzt) : 0.0);
        }
  }
  // per-plane z tables of every box (ZJ_*): constants on a uniform axis
  for (size_t bi = 0; bi < c->h_boxes.size(); ++bi) {
    BoxDev& d = c->h_boxes[bi];
    d.joff = (long long)ztab.size();
    const bool cst = p->nu_const > 0.0;
    for (int k = 0; k < d.nzt; ++k) {
      double jc = 1.0 / d.dz, jf = 1.0 / d.dz, dc = d.dz, df = d.dz;
      if (d.stretched) {
        // the wall end copy: the up output at the top plane and the down
        // output at the bottom plane take their neighbour's stencil
        const int kc = k == d.nzt - 1 ? k - 1 : k, kf = k == 0 ? 1 : k;
        jc = 1.0 / c->dzc[bi][kc];
        jf = 1.0 / c->dzf[bi][kf];
        dc = c->dzc[bi][k];
        df = c->dzf[bi][k];
      }
      double e[ZJ_COUNT];
      e[ZJ_C] = jc;
      e[ZJ_F] = jf;
      e[ZJ_LZZ] = cst ? d.hmin : (d.stretched ? dc : d.lv[2]);
      e[ZJ_LXZ] = cst ? d.hmin : (d.stretched ? std::max(d.dx, df) : d.le[1]);
      e[ZJ_LYZ] = cst ? d.hmin : (d.stretched ? std::max(d.dy, df) : d.le[2]);
      e[ZJ_LZF] = cst ? d.hmin : (d.stretched ? df : d.lv[2]);
      e[ZJ_H] = cst ? d.hmin : (d.stretched ? std::min(std::min(d.dx, d.dy), dc) : d.hmin);
      e[ZJ_DZC] = dc;
      for (int q = 0; q < ZJ_COUNT; ++q) ztab.push_back(e[q]);
    }
  }
  std::vector<Blk> tab, gtab;
  build_tables(c, tab, gtab);
  c->nblk = (int)tab.size();
  c->ngblk = (int)gtab.size();
  hipError_t e;
  if ((e = hipMalloc(&c->d_boxes, sizeof(BoxDev) * c->h_boxes.size())) != hipSuccess ||
      (e = hipMalloc(&c->d_tab, sizeof(Blk) * tab.size())) != hipSuccess ||
      (c->ngblk && (e = hipMalloc(&c->d_gtab, sizeof(Blk) * gtab.size())) != hipSuccess) ||
      (e = hipMalloc(&c->d_tot, sizeof(RedTotal))) != hipSuccess ||
      (e = hipMalloc(&c->work, (size_t)work_arrays(c->p) * c->nelem * c->esize)) != hipSuccess) {
    g_init_err = std::string("device allocation failed: ") + hipGetErrorString(e);
    mhd_destroy(c);
    return MHD_ENOMEM;
  }
  if ((e = hipMemcpy(c->d_boxes, c->h_boxes.data(), sizeof(BoxDev) * c->h_boxes.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->d_tab, tab.data(), sizeof(Blk) * tab.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (c->ngblk && (e = hipMemcpy(c->d_gtab, gtab.data(), sizeof(Blk) * gtab.size(), hipMemcpyHostToDevice)) != hipSuccess)) {
    g_init_err = std::string("table upload failed: ") + hipGetErrorString(e);
    mhd_destroy(c);
    return MHD_EHIP;
  }
  if (!ztab.empty()) {
    const size_t nb = ztab.size() * c->esize;
    if ((e = hipMalloc(&c->d_ztab, nb)) != hipSuccess) {
      g_init_err = std::string("device allocation failed: ") + hipGetErrorString(e);
      mhd_destroy(c);
      return MHD_ENOMEM;
    }
    std::vector<float> zf(ztab.begin(), ztab.end());
    e = hipMemcpy(c->d_ztab, c->esize == 4 ? (const void*)zf.data() : (const void*)ztab.data(), nb,
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      g_init_err = std::string("table upload failed: ") + hipGetErrorString(e);
      mhd_destroy(c);
      return MHD_EHIP;
    }
  }
  if ((e = hipMalloc(&c->d_dt, sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&c->d_queue, sizeof(int) * kQueueInts)) != hipSuccess ||
      (e = hipMalloc(&c->d_lnavg, c->esize * (size_t)c->nplanes)) != hipSuccess ||
      (e = hipMalloc(&c->d_lnpart, sizeof(double) * kPlaneSlices * (size_t)c->nplanes)) != hipSuccess ||
      (e = hipMalloc(&c->d_lnpav, c->esize * (size_t)c->nplanes)) != hipSuccess) {
    g_init_err = std::string("device allocation failed: ") + hipGetErrorString(e);
    mhd_destroy(c);
    return MHD_ENOMEM;
  }
  // float64 kernels hold twice the data per column: smaller default tile
  const int tile = p->dtype == MHD_F64 ? ZTILE_16x8 : ZTILE_32x8;
  if (set_tile(c, tile) != MHD_OK) {
    g_init_err = c->err;
    mhd_destroy(c);
    return MHD_ENOMEM;
  }
  *out = c;
  return MHD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
template <class T>
static ZStageArgs<T> zargs(mhd_ctx* c, const Scratch& s) {
  ZStageArgs<T> a;
  a.w = make_zwork<T>(c, s);
  a.ph = make_phys<T>(c->p);
  a.du = p8null<T>();
  a.du_mode = 0;
  a.f_out = p8null<T>();
  a.alpha = T(0);
  a.beta = 0.0;
  a.dt_dev = nullptr;
  a.dt_host = 0.0;
  a.cpart = nullptr;
  a.ztab = static_cast<const T*>(c->d_ztab);
  a.lnavg = static_cast<T*>(s.lnavg);
  a.lnpart = s.lnpart;
  a.Cdt = c->p.Cdt;
  a.Cdtd = c->p.Cdtd;
  a.nuB = c->p.nuB;
  a.eta_const = c->p.eta_const;
  return a;
}
template <class T> static ZStageArgs<T> zargs(mhd_ctx* c) { return zargs<T>(c, own_scratch(c)); }

template <class T>
static int do_rhs(mhd_ctx* c, void* const f[8], void* const dfdt[8], const Scratch& s) {
  const Launch L = make_launch(c);
  launch_ghost<T>(L, p8<T>(f));
  ZStageArgs<T> a = zargs<T>(c, s);
  a.f = cp8<T>(f);
  a.du = p8<T>(dfdt);
  launch_zstage<T>(make_zlaunch(c, s), a);
  return check_launch(c, "mhd_rhs launch");
}

// One RK stage of the middle form (reads f and dU, writes dU and the next
// state, the most bytes of the three), as the autotuner times it: the
// shape that is fastest for a bare right-hand side need not be fastest for
// the stages of a step, whose pass F also streams dU and the states.
template <class T>
static void autotune_stage(mhd_ctx* c, void* const f[8], void* const du[8], void* next) {
  ZStageArgs<T> a = zargs<T>(c);
  a.f = cp8<T>(f);
  a.du = p8<T>(du);
  a.du_mode = DU_READ | DU_WRITE;
  P8<T> o;
  for (int v = 0; v < 8; ++v) o.p[v] = static_cast<T*>(next) + (long long)v * c->nelem;
  a.f_out = o;
  a.alpha = T(kAlpha[1]);
  a.beta = kBeta[1];
  a.dt_host = 1e-12;
  launch_zstage<T>(make_zlaunch(c), a);
}

// dt > 0: fixed step.  dt == 0: the Courant step of each step's initial
// state, computed on the device during the first stage (never leaves it).
template <class T>
static int do_step(mhd_ctx* c, void* const f[8], void* const t1[8], void* const t2[8],
                   void* const du[8], double dt, int nsteps) {
  const Launch L = make_launch(c);
  const ZLaunch Z = make_zlaunch(c);
  const P8<T> F = p8<T>(f), A = p8<T>(t1), B = p8<T>(t2), U = p8<T>(du);
  const bool cfl = dt == 0.0;
  launch_ghost<T>(L, F);
  for (int n = 0; n < nsteps; ++n) {
    // stage states: f -> t1 -> t2 -> f (the stage input is never written)
    const P8<T> src[3] = {F, A, B};
    const P8<T> dst[3] = {A, B, F};
    for (int s = 0; s < 3; ++s) {
      ZStageArgs<T> a = zargs<T>(c);
      a.f = cp8<T>(src[s]);
      a.du = U;
      a.du_mode = (s == 0 ? 0 : DU_READ) | (s == 2 ? 0 : DU_WRITE);
      a.f_out = dst[s];
      a.alpha = T(kAlpha[s]);
      a.beta = kBeta[s];
      a.dt_host = dt;
      if (cfl) {
        a.dt_dev = c->d_dt;
        if (s == 0) a.cpart = c->d_cpart;
      }
      launch_zstage<T>(Z, a);
      launch_ghost<T>(L, dst[s]);
    }
  }
  return check_launch(c, "mhd_step launch");
}

// The right-hand side as a planned program, built once per context, and
// again when the div B diffusion's dt changes (dt 0: without that term).
static int ensure_program(mhd_ctx* c, double dt) {
  if (!(c->p.terms & MHD_T_DIVB)) dt = 0.0;
  if (c->prog && c->prog_dt == dt) return MHD_OK;
  if (c->prog) {
    delete c->prog;
    c->prog = nullptr;
    (void)hipFree(c->d_fused);
    (void)hipFree(c->d_bsteps);
    c->d_fused = nullptr;
    c->d_bsteps = nullptr;
  }
  if (!c->d_pm && hipMalloc(&c->d_pm, sizeof(double) * std::max(1, c->nplanes)) != hipSuccess)
    return fail(c, MHD_ENOMEM, "adjoint plane means");
  VPlan* P = nullptr;
  try {
    P = new VPlan(plan_program(build_rhs_program(c->p, dt)));
  } catch (...) {
    return fail(c, MHD_ENOMEM, "adjoint program");
  }
  const size_t bytes = sizeof(VFused) * P->fused.size(), bbytes = sizeof(VStep) * P->bsteps.size();
  hipError_t e = hipMalloc(&c->d_fused, bytes);
  if (e == hipSuccess) e = hipMemcpy(c->d_fused, P->fused.data(), bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&c->d_bsteps, bbytes);
  if (e == hipSuccess) e = hipMemcpy(c->d_bsteps, P->bsteps.data(), bbytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(c->d_fused);
    (void)hipFree(c->d_bsteps);
    c->d_fused = nullptr;
    c->d_bsteps = nullptr;
    delete P;
    return fail(c, MHD_ENOMEM, "adjoint program upload");
  }
  c->prog = P;
  c->prog_dt = dt;
  return MHD_OK;
}

// Adjoint of one RK step (dt fixed).  With f_s the stage inputs, U_s the
// 2N-storage derivative and F_s = F(f_s):
//   U_s = alpha_s U_{s-1} + F_s,  f_{s+1} = f_s + beta_s dt U_s,
// so, backwards from gbar = gbar_in (the cotangent of f_3):
//   Ubar_s = alpha_{s+1} Ubar_{s+1} + beta_s dt gbar,
//   gbar  += (dF/df at f_s)^T Ubar_s.
// f_1 and f_2 come from the fused stage kernels; F's intermediates at each
// f_s from the program's forward run, just before its transpose.
static VLaunch make_vlaunch(mhd_ctx* c) {
  return VLaunch{c->d_boxes, c->d_tab, c->nblk, c->stream, (int)c->h_boxes.size(), c->nplanes, c->d_pm,
                 c->d_ztab, c->d_gtab, c->ngblk};
}

static bool any_wall(const mhd_ctx* c) {
  for (const auto& b : c->boxes)
    if (b.bc_z == MHD_BC_WALL) return true;
  return false;
}

// The adjoint workspace: the program's value and cotangent slots, then the
// stage states and dU (25 arrays; 16 more with walls: the filled input and
// the step's end state).
template <class T> static T* adjoint_workspace(mhd_ctx* c, const VPlan& P, bool walls, int& rc) {
  const long long n = c->nelem;
  const size_t narr = (size_t)P.nval + P.ncot + 25 + (walls ? 16 : 0);
  const size_t need = narr * (size_t)n * c->esize;
  rc = MHD_OK;
  if (c->adj_bytes < need) {
    (void)hipFree(c->adj);
    c->adj = nullptr;
    c->adj_bytes = 0;
    if (hipMalloc(&c->adj, need) != hipSuccess) {
      rc = fail(c, MHD_ENOMEM, "adjoint workspace");
      return nullptr;
    }
    c->adj_bytes = need;
  }
  return static_cast<T*>(c->adj);
}

// One RK step's adjoint at fixed dt.  The stage states are recomputed with
// the stage kernels; then, stage by stage backwards, Ubar = alpha Ubar +
// beta dt G, the program's forward run at the stage state and its reverse
// sweep seeded with Ubar give G += (dF/df)^T Ubar.  With walls the states
// are filled (the step fills before every F and after the last stage),
// Ubar is masked like F, and G passes through the fill's transpose after
// each stage (and first through that of the end state's fill).
template <class T>
static int do_adjoint(mhd_ctx* c, void* const fn[8], double dt, void* const gin[8],
                      void* const gout[8]) {
  if (int rc = ensure_program(c, dt)) return rc;
  const VPlan& P = *c->prog;
  const long long n = c->nelem;
  const bool walls = any_wall(c);
  int rc = MHD_OK;
  T* base = adjoint_workspace<T>(c, P, walls, rc);
  if (!base) return rc;
  T* cbase = base + (long long)P.nval * n;
  T* rest = cbase + (long long)P.ncot * n;
  auto set8 = [&](int first) {
    P8<T> q;
    for (int v = 0; v < 8; ++v) q.p[v] = rest + (long long)(first + v) * n;
    return q;
  };
  const P8<T> F1 = set8(0), F2 = set8(8), U = set8(16);
  const P8<T> S0 = walls ? set8(25) : p8<T>(fn), F3 = set8(walls ? 33 : 0);
  const P8<T> G = p8<T>(gout);
  const size_t bytes = (size_t)n * c->esize;
  T* zeros = rest + 24LL * n;   // the cotangent of an input F does not read
  const Launch L = make_launch(c);
  hipError_t e = hipSuccess;
  if (walls) {
    // the step fills its input first; f_n itself is left as it is
    for (int v = 0; v < 8 && e == hipSuccess; ++v)
      e = hipMemcpyAsync(S0.p[v], fn[v], bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return fail(c, MHD_EHIP, hipGetErrorString(e));
    launch_ghost<T>(L, S0);
  }
  // stage states f_1, f_2 (and with walls the end state, for its fill)
  const ZLaunch Z = make_zlaunch(c);
  for (int s = 0; s < (walls ? 3 : 2); ++s) {
    ZStageArgs<T> a = zargs<T>(c);
    a.f = s == 0 ? cp8<T>(S0) : (s == 1 ? cp8<T>(F1) : cp8<T>(F2));
    a.du = U;
    a.du_mode = (s == 0 ? 0 : DU_READ) | (s == 2 ? 0 : DU_WRITE);
    a.f_out = s == 0 ? F1 : (s == 1 ? F2 : F3);
    a.alpha = T(kAlpha[s]);
    a.beta = kBeta[s];
    a.dt_host = dt;
    launch_zstage<T>(Z, a);
    if (walls) launch_ghost<T>(L, a.f_out);
  }
  L.at(PASS_ADJOINT);
  const VLaunch V = make_vlaunch(c);
  e = hipMemsetAsync(zeros, 0, bytes, c->stream);
  for (int v = 0; v < 8 && e == hipSuccess; ++v)
    e = hipMemcpyAsync(G.p[v], gin[v], bytes, hipMemcpyDeviceToDevice, c->stream);
  // (value slots are free outside the program's runs: the fill's transpose
  // keeps its temporaries there)
  if (walls && e == hipSuccess) vm_fill_vjp<T>(V, cp8<T>(F3), G, base, n);
  const P8<T> Ub = U;   // U is free again: it becomes Ubar
  for (int s = 2; s >= 0 && e == hipSuccess; --s) {
    vm_axpby8<T>(V, Ub, cp8<T>(G), s == 2 ? 0.0 : kAlpha[s + 1], kBeta[s] * dt);
    if (walls) vm_wall_mask<T>(V, Ub);
    const P8<T> fs = s == 0 ? S0 : (s == 1 ? F1 : F2);
    for (int v = 0; v < 8 && e == hipSuccess; ++v)
      e = hipMemcpyAsync(base + (long long)v * n, fs.p[v], bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) break;
    vm_forward<T>(V, P, c->d_fused, base, n);
    for (int v = 0; v < 8 && e == hipSuccess; ++v)
      e = hipMemcpyAsync(cbase + (long long)P.cout[v] * n, Ub.p[v], bytes, hipMemcpyDeviceToDevice,
                         c->stream);
    if (e != hipSuccess) break;
    vm_backward<T>(V, P, c->d_bsteps, base, cbase, n);
    CP8<T> cin;
    bool any = false;
    for (int v = 0; v < 8; ++v) {
      cin.p[v] = P.cin[v] >= 0 ? cbase + (long long)P.cin[v] * n : zeros;
      any |= P.cin[v] >= 0;
    }
    if (any) vm_axpby8<T>(V, G, cin, 1.0, 1.0);
    if (walls) vm_fill_vjp<T>(V, cp8<T>(fs), G, base, n);
  }
  L.at(PASS_END);
  if (e != hipSuccess) return fail(c, MHD_EHIP, hipGetErrorString(e));
  return check_launch(c, "mhd_step_adjoint launch");
}

// (dF/df)^T wbar at the state f: the program's forward run at f, its
// reverse sweep seeded with wbar.  With walls, F is the right-hand side of
// mhd_rhs, which fills the ghost planes first: the run is at the filled
// state, the seed is masked like F, and the result passes through the
// fill's transpose.
template <class T>
static int do_rhs_adjoint(mhd_ctx* c, void* const f[8], void* const wbar[8],
                          void* const fbar[8]) {
  if (int rc = ensure_program(c, 0.0)) return rc;
  const VPlan& P = *c->prog;
  const long long n = c->nelem;
  const bool walls = any_wall(c);
  int rc = MHD_OK;
  T* base = adjoint_workspace<T>(c, P, walls, rc);
  if (!base) return rc;
  T* cbase = base + (long long)P.nval * n;
  T* rest = cbase + (long long)P.ncot * n;
  const size_t bytes = (size_t)n * c->esize;
  const Launch L = make_launch(c);
  L.at(PASS_ADJOINT);
  const VLaunch V = make_vlaunch(c);
  P8<T> S, W;
  for (int v = 0; v < 8; ++v) {
    S.p[v] = rest + (long long)v * n;          // the filled state (walls)
    W.p[v] = rest + (long long)(8 + v) * n;    // the masked seed (walls)
  }
  hipError_t e = hipSuccess;
  for (int v = 0; v < 8 && e == hipSuccess; ++v)
    e = hipMemcpyAsync(base + (long long)v * n, f[v], bytes, hipMemcpyDeviceToDevice, c->stream);
  if (walls) {
    for (int v = 0; v < 8 && e == hipSuccess; ++v) {
      e = hipMemcpyAsync(S.p[v], f[v], bytes, hipMemcpyDeviceToDevice, c->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(W.p[v], wbar[v], bytes, hipMemcpyDeviceToDevice, c->stream);
    }
    if (e == hipSuccess) {
      launch_ghost<T>(L, S);
      vm_wall_mask<T>(V, W);
    }
    for (int v = 0; v < 8 && e == hipSuccess; ++v)
      e = hipMemcpyAsync(base + (long long)v * n, S.p[v], bytes, hipMemcpyDeviceToDevice, c->stream);
  }
  if (e == hipSuccess) vm_forward<T>(V, P, c->d_fused, base, n);
  for (int v = 0; v < 8 && e == hipSuccess; ++v)
    e = hipMemcpyAsync(cbase + (long long)P.cout[v] * n, walls ? W.p[v] : wbar[v], bytes,
                       hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) vm_backward<T>(V, P, c->d_bsteps, base, cbase, n);
  for (int v = 0; v < 8 && e == hipSuccess; ++v)
    e = P.cin[v] >= 0 ? hipMemcpyAsync(fbar[v], cbase + (long long)P.cin[v] * n, bytes,
                                       hipMemcpyDeviceToDevice, c->stream)
                      : hipMemsetAsync(fbar[v], 0, bytes, c->stream);
  if (walls && e == hipSuccess) vm_fill_vjp<T>(V, cp8<T>(S), p8<T>(fbar), base, n);
  L.at(PASS_END);
  if (e != hipSuccess) return fail(c, MHD_EHIP, hipGetErrorString(e));
  return check_launch(c, "mhd_rhs_adjoint launch");
}

template <class T>
static int do_reduce(mhd_ctx* c, void* const f[8], void* const dfdt[8], mhd_stats* out) {
  const Launch L = make_launch(c);
  launch_ghost<T>(L, p8<T>(f));
  const ZLaunch Z = make_zlaunch(c);
  Z.at(PASS_REDUCE);
  launch_zreduce<T>(Z, cp8<T>(f), cp8<T>(dfdt), make_zwork<T>(c), make_phys<T>(c->p),
                    static_cast<const T*>(c->d_ztab), c->d_red, c->d_tot, c->p.Cdt, c->p.Cdtd, c->p.Cdtr,
                    c->p.nuB, c->p.eta_const);
  Z.at(PASS_END);
  int rc = check_launch(c, "mhd_reductions launch");
  if (rc) return rc;
  RedTotal tot;
  hipError_t e = hipMemcpyAsync(&tot, c->d_tot, sizeof(RedTotal), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hipfail(c, e, "mhd_reductions readback");
  memset(out, 0, sizeof(*out));
  out->mass = tot.sum[0];
  out->mom[0] = tot.sum[1];
  out->mom[1] = tot.sum[2];
  out->mom[2] = tot.sum[3];
  out->ekin = tot.sum[4];
  out->emag = tot.sum[5] / (2.0 * c->p.mu);
  out->eint = tot.sum[6];
  long long ninter = 0;
  for (const auto& b : c->boxes) ninter += (long long)b.nx * b.ny * b.nz;
  out->divb_max = tot.mx[0];
  out->divb_rms = std::sqrt(tot.sum[7] / (double)ninter);
  out->bmax = tot.mx[1];
  out->umax = tot.mx[2];
  out->cmax = tot.cmax;
  out->numax = tot.dmax;
  out->ratemax = dfdt ? tot.rmax : 0.0;
  const double inf = std::numeric_limits<double>::infinity();
  out->dt_wave = tot.dtw;
  out->dt_diff = tot.dtd;
  out->dt_rate = dfdt ? tot.dtr : inf;
  long long arg = tot.warg;
  out->dt = out->dt_wave;
  out->dt_limit = 0;
  if (out->dt_diff < out->dt) { out->dt = out->dt_diff; out->dt_limit = 1; arg = tot.darg; }
  if (out->dt_rate < out->dt) { out->dt = out->dt_rate; out->dt_limit = 2; arg = tot.rarg; }
  int box = 0;
  for (int b = 0; b < (int)c->offsets.size(); ++b)
    if (arg >= c->offsets[b]) box = b;
  out->dt_box = box;
  out->dt_argmax = arg - c->offsets[box];
  out->n_nonfinite = tot.nonfinite;
  out->n_nonpositive = tot.nonpositive;
  if (tot.nonfinite || tot.nonpositive) {
    c->err = "non-finite or non-positive state";
    return MHD_ENONFINITE;
  }
  return MHD_OK;
}

extern "C" {

int mhd_rhs(mhd_ctx* c, void* const f[8], void* const dfdt[8]) {
  if (!c) return fail(nullptr, MHD_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = check8(c, f, "f")) || (rc = check8(c, dfdt, "dfdt"))) return rc;
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b)
      if (f[a] == dfdt[b]) return fail(c, MHD_EINVAL, "f and dfdt overlap");
  return c->p.dtype == MHD_F32 ? do_rhs<float>(c, f, dfdt, own_scratch(c))
                               : do_rhs<double>(c, f, dfdt, own_scratch(c));
}

// Layout of a context's per-call scratch inside the static array: returns
// the bytes it needs, and fills *s only when they fit.
static size_t static_layout(const mhd_ctx* c, Scratch* s) {
  auto a256 = [](size_t n) { return (n + 255) & ~size_t(255); };
  const size_t work = a256((size_t)work_arrays(c->p) * c->nelem * c->esize);
  const size_t tab = a256(c->esize * (size_t)c->nplanes);
  const size_t part = a256(sizeof(double) * kPlaneSlices * (size_t)c->nplanes);
  const size_t need = work + 2 * tab + part + a256(sizeof(int) * kQueueInts);
  if (s && c->scratch && need <= kScratchBytes) {
    char* b = static_cast<char*>(c->scratch);
    *s = Scratch{b, b + work, b + work + tab, reinterpret_cast<double*>(b + work + 2 * tab),
                 reinterpret_cast<int*>(b + work + 2 * tab + part)};
  }
  return need;
}

int mhd_rhs_noalloc(mhd_ctx* c, void* const f[8], void* const dfdt[8]) {
  if (!c) return fail(nullptr, MHD_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = check8(c, f, "f")) || (rc = check8(c, dfdt, "dfdt"))) return rc;
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b)
      if (f[a] == dfdt[b]) return fail(c, MHD_EINVAL, "f and dfdt overlap");
  if (!c->scratch) return fail(c, MHD_EHIP, "mhd_rhs_noalloc: the static scratch is not available on this device");
  Scratch s;
  const size_t need = static_layout(c, &s);
  if (need > kScratchBytes)
    return fail(c, MHD_EINVAL, "mhd_rhs_noalloc: these boxes need " + std::to_string(need) +
                                   " bytes of scratch, above the static limit of " +
                                   std::to_string(kScratchBytes) + " bytes (use mhd_rhs)");
  return c->p.dtype == MHD_F32 ? do_rhs<float>(c, f, dfdt, s) : do_rhs<double>(c, f, dfdt, s);
}

int mhd_step(mhd_ctx* c, void* const f[8], void* const t1[8], void* const t2[8],
             void* const du[8], double dt, int32_t nsteps) {
  if (!c) return fail(nullptr, MHD_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = check8(c, f, "f")) || (rc = check8(c, t1, "tmp1")) || (rc = check8(c, t2, "tmp2")) ||
      (rc = check8(c, du, "dU")))
    return rc;
  if (nsteps < 0) return fail(c, MHD_EINVAL, "nsteps < 0");
  if (!std::isfinite(dt) || dt < 0.0) return fail(c, MHD_EINVAL, "dt must be finite and >= 0");
  void* const* sets[4] = {f, t1, t2, du};
  for (int x = 0; x < 4; ++x)
    for (int y = x + 1; y < 4; ++y)
      for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b)
          if (sets[x][a] == sets[y][b]) return fail(c, MHD_EINVAL, "state, temporaries and dU must not overlap");
  if (nsteps == 0) return MHD_OK;
  return c->p.dtype == MHD_F32 ? do_step<float>(c, f, t1, t2, du, dt, nsteps)
                               : do_step<double>(c, f, t1, t2, du, dt, nsteps);
}

int mhd_reductions(mhd_ctx* c, void* const f[8], void* const dfdt[8], mhd_stats* out) {
  if (!c) return fail(nullptr, MHD_EINVAL, "ctx is NULL");
  if (!out) return fail(c, MHD_EINVAL, "out is NULL");
  int rc;
  if ((rc = check8(c, f, "f"))) return rc;
  if (dfdt && (rc = check8(c, dfdt, "dfdt"))) return rc;
  return c->p.dtype == MHD_F32 ? do_reduce<float>(c, f, dfdt, out)
                               : do_reduce<double>(c, f, dfdt, out);
}

int mhd_divb_clean(mhd_ctx* c, void* const f[8]) {
  if (!c) return fail(nullptr, MHD_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = check8(c, f, "f"))) return rc;
  for (const auto& b : c->boxes)
    if (b.bc_z != MHD_BC_PERIODIC)
      return fail(c, MHD_EUNSUPPORTED, "div B cleaning in Fourier space needs periodic boxes");
  std::string err;
  const int r = c->p.dtype == MHD_F32 ? clean_boxes<float>(&c->clean, c->h_boxes, p8<float>(f), c->stream, err)
                                      : clean_boxes<double>(&c->clean, c->h_boxes, p8<double>(f), c->stream, err);
  if (r == 2) return fail(c, MHD_ENOMEM, "mhd_divb_clean: " + err);
  if (r) return fail(c, MHD_EHIP, "mhd_divb_clean: " + err);
  return check_launch(c, "mhd_divb_clean launch");
}

int mhd_step_adjoint(mhd_ctx* c, void* const f_n[8], double dt, void* const gin[8],
                     void* const gout[8]) {
  if (!c) return fail(nullptr, MHD_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = check8(c, f_n, "f_n")) || (rc = check8(c, gin, "gbar_in")) ||
      (rc = check8(c, gout, "gbar_out")))
    return rc;
  if (!std::isfinite(dt) || !(dt > 0.0)) return fail(c, MHD_EINVAL, "dt must be finite and > 0");
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b)
      if (gin[a] == gout[b] || f_n[a] == gout[b]) return fail(c, MHD_EINVAL, "gbar_out overlaps an input");
  return c->p.dtype == MHD_F32 ? do_adjoint<float>(c, f_n, dt, gin, gout)
                               : do_adjoint<double>(c, f_n, dt, gin, gout);
}

int mhd_rhs_adjoint(mhd_ctx* c, void* const f[8], void* const wbar[8], void* const fbar[8]) {
  if (!c) return fail(nullptr, MHD_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = check8(c, f, "f")) || (rc = check8(c, wbar, "wbar")) || (rc = check8(c, fbar, "fbar")))
    return rc;
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b)
      if (fbar[b] == f[a] || fbar[b] == wbar[a]) return fail(c, MHD_EINVAL, "fbar overlaps an input");
  return c->p.dtype == MHD_F32 ? do_rhs_adjoint<float>(c, f, wbar, fbar)
                               : do_rhs_adjoint<double>(c, f, wbar, fbar);
}

int mhd_profile(mhd_ctx* c, int32_t enable) {
  if (!c) return fail(nullptr, MHD_EINVAL, "ctx is NULL");
  int rc = prof_fold(c);
  for (int q = 0; q < PASS_COUNT; ++q) {
    c->prof_ms[q] = 0.0;
    c->prof_n[q] = 0;
  }
  c->prof = enable != 0;
  return rc ? fail(c, rc, "profile reset: event timing failed") : MHD_OK;
}

int mhd_profile_read(mhd_ctx* c, double* ms, int64_t* count, int32_t n) {
  if (!c) return fail(nullptr, MHD_EINVAL, "ctx is NULL");
  if (!ms || !count || n < 0) return fail(c, MHD_EINVAL, "bad output arrays");
  int rc = prof_fold(c);
  if (rc) return fail(c, rc, "profile read: event timing failed");
  for (int q = 0; q < n && q < PASS_COUNT; ++q) {
    ms[q] = c->prof_ms[q];
    count[q] = c->prof_n[q];
  }
  return MHD_OK;
}

int mhd_last_dt(mhd_ctx* c, double* dt) {
  if (!c) return fail(nullptr, MHD_EINVAL, "ctx is NULL");
  if (!dt) return fail(c, MHD_EINVAL, "dt is NULL");
  hipError_t e = hipMemcpyAsync(dt, c->d_dt, sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? MHD_OK : hipfail(c, e, "mhd_last_dt");
}

int mhd_set_tile(mhd_ctx* c, int32_t tile) {
  if (!c) return fail(nullptr, MHD_EINVAL, "ctx is NULL");
  if (tile < 0 || tile >= ZTILE_COUNT) return fail(c, MHD_EINVAL, "unknown tile shape");
  if (!ztile_ok(tile, c->esize)) return fail(c, MHD_EUNSUPPORTED, "tile shape not built for this dtype");
  return set_tile(c, tile);
}

int mhd_set_launch(mhd_ctx* c, int32_t tile, int32_t persistent) {
  if (!c) return fail(nullptr, MHD_EINVAL, "ctx is NULL");
  if (tile < 0 || tile >= ZTILE_COUNT) return fail(c, MHD_EINVAL, "unknown tile shape");
  if (persistent != 0 && persistent != 1) return fail(c, MHD_EINVAL, "persistent must be 0 or 1");
  if (!ztile_ok(tile, c->esize)) return fail(c, MHD_EUNSUPPORTED, "tile shape not built for this dtype");
  int rc = set_tile(c, tile);
  if (rc == MHD_OK) c->persistent = persistent;
  return rc;
}

int mhd_get_launch(const mhd_ctx* c, int32_t* tile, int32_t* persistent) {
  if (!c || !tile || !persistent) return MHD_EINVAL;
  *tile = c->tile;
  *persistent = c->persistent;
  return MHD_OK;
}

int mhd_set_final_tile(mhd_ctx* c, int32_t tile) {
  if (!c) return fail(nullptr, MHD_EINVAL, "ctx is NULL");
  if (tile < 0 || tile >= ZTILE_COUNT) return fail(c, MHD_EINVAL, "unknown tile shape");
  if (!ztile_ok(tile, c->esize)) return fail(c, MHD_EUNSUPPORTED, "tile shape not built for this dtype");
  return set_ftile(c, tile);
}

int mhd_get_final_tile(const mhd_ctx* c, int32_t* tile) {
  if (!c || !tile) return MHD_EINVAL;
  *tile = c->ftile;
  return MHD_OK;
}

int mhd_autotune(mhd_ctx* c, void* const f[8], void* const dfdt[8], int32_t reps, double* ms) {
  if (!c) return fail(nullptr, MHD_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = check8(c, f, "f")) || (rc = check8(c, dfdt, "dfdt"))) return rc;
  if (reps < 1) return fail(c, MHD_EINVAL, "reps < 1");
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b)
      if (f[a] == dfdt[b]) return fail(c, MHD_EINVAL, "f and dfdt overlap");
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(c, MHD_EHIP, "event");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(c, MHD_EHIP, "event");
  }
  // the next state of the timed stages (freed before returning)
  void* next = nullptr;
  if (hipMalloc(&next, (size_t)8 * c->nelem * c->esize) != hipSuccess) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return fail(c, MHD_ENOMEM, "autotune scratch");
  }
  const bool prof = c->prof;
  c->prof = false;
  // milliseconds per RK stage in the current launch configuration
  auto timed = [&](double& per) {
    int r0 = mhd_rhs(c, f, dfdt);   // warm-up (and, with walls, the ghost fill); dU = F
    (void)hipEventRecord(e0, c->stream);
    for (int r = 0; r < reps && r0 == MHD_OK; ++r) {
      if (c->p.dtype == MHD_F32) autotune_stage<float>(c, f, dfdt, next);
      else autotune_stage<double>(c, f, dfdt, next);
      r0 = check_launch(c, "autotune stage");
    }
    (void)hipEventRecord(e1, c->stream);
    float el = 0.0f;
    if (r0 == MHD_OK && (hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&el, e0, e1) != hipSuccess))
      r0 = fail(c, MHD_EHIP, "autotune timing");
    per = (double)el / reps;
    return r0;
  };
  // every pass in one shape and mode.  Each candidate is timed in
  // kRounds rounds over all candidates and keeps its fastest: a launch's
  // time varies from call to call by several percent (the memory system's
  // state), more than some candidates differ.
  constexpr int kRounds = 3;
  double tm[ZTILE_COUNT][2];
  for (int t = 0; t < ZTILE_COUNT; ++t) tm[t][0] = tm[t][1] = -1.0;
  for (int round = 0; round < kRounds && rc == MHD_OK; ++round)
    for (int t = 0; t < ZTILE_COUNT && rc == MHD_OK; ++t)
      for (int m = 0; m < 2 && rc == MHD_OK; ++m) {
        if (!ztile_ok(t, c->esize)) continue;
        if ((rc = mhd_set_launch(c, t, m)) != MHD_OK) break;
        double per = 0.0;
        rc = timed(per);
        if (rc == MHD_OK && (tm[t][m] < 0.0 || per < tm[t][m])) tm[t][m] = per;
      }
  double best = -1.0;
  int bt = c->tile, bp = c->persistent;
  for (int t = 0; t < ZTILE_COUNT; ++t)
    for (int m = 0; m < 2; ++m) {
      if (ms) ms[t * 2 + m] = tm[t][m] > 0.0 ? tm[t][m] : 0.0;
      if (tm[t][m] > 0.0 && (best < 0.0 || tm[t][m] < best)) {
        best = tm[t][m];
        bt = t;
        bp = m;
      }
    }
  // then pass F's own shape, with the others' shape fixed, in both modes
  // (fastest of the rounds again): a change only if it is faster by more
  // than the timing noise (1 %; the fastest of three rounds varies by about
  // 0.1 %)
  double tf[2][ZTILE_COUNT];
  for (int m = 0; m < 2; ++m)
    for (int t = 0; t < ZTILE_COUNT; ++t) tf[m][t] = -1.0;
  for (int round = 0; round < kRounds && rc == MHD_OK; ++round)
    for (int m = 0; m < 2 && rc == MHD_OK; ++m) {
      if ((rc = mhd_set_launch(c, bt, m)) != MHD_OK) break;
      for (int t = 0; t < ZTILE_COUNT && rc == MHD_OK; ++t) {
        if (!ztile_ok(t, c->esize)) continue;
        if ((rc = set_ftile(c, t)) != MHD_OK) break;
        double per = 0.0;
        rc = timed(per);
        if (rc == MHD_OK && (tf[m][t] < 0.0 || per < tf[m][t])) tf[m][t] = per;
      }
    }
  int bm = bp, bf = bt;
  if (rc == MHD_OK) {
    const double base = tf[bp][bt];
    for (int m = 0; m < 2; ++m)
      for (int t = 0; t < ZTILE_COUNT; ++t)
        if (tf[m][t] > 0.0 && tf[m][t] < 0.99 * base && tf[m][t] < tf[bm][bf]) {
          bm = m;
          bf = t;
        }
    rc = mhd_set_launch(c, bt, bm);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(next);
  c->prof = prof;
  if (rc != MHD_OK) return rc;
  return set_ftile(c, bf);
}

}  // extern "C"
