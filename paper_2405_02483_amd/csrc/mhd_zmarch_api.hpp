// Host-side view of the z-marching stage kernels (mhd_zmarch.hip).
#pragma once

#include "mhd_zmarch.hpp"

namespace smhd {

// Outputs of pass Q, in workspace order.
enum QOut : int {
  QOUT_GXZ = 0, QOUT_GZX, QOUT_EY, QOUT_LXY, QOUT_LZY, QOUT_QY,
  QOUT_GYZ, QOUT_GZY, QOUT_EX, QOUT_LYX, QOUT_LZX, QOUT_QX,
  QOUT_HZ, QOUT_GZZ, QOUT_CZZ, QOUT_DPZ, QOUT_COUNT
};

template <class T> struct QP { T* p[QOUT_COUNT]; };
template <class T> struct CQP { const T* p[QOUT_COUNT]; };

// Outputs of pass P, in workspace order.
enum POut : int {
  POUT_GXY = 0, POUT_GYX, POUT_EZ, POUT_LXZ, POUT_LYZ, POUT_QZ,
  POUT_GXX, POUT_GYY, POUT_QC, POUT_HX, POUT_HY, POUT_DPX, POUT_DPY, POUT_COUNT
};

template <class T> struct PQ { T* p[POUT_COUNT]; };
template <class T> struct CPQ { const T* p[POUT_COUNT]; };

// Tile shapes (columns per workgroup, x by y) the stage kernels are built for.
enum ZTile : int {
  ZTILE_64x4 = 0, ZTILE_32x8 = 1, ZTILE_16x16 = 2, ZTILE_16x8 = 3, ZTILE_64x8 = 4, ZTILE_32x16 = 5, ZTILE_COUNT
};

// Whether a tile shape is built for an element size (all are).
inline bool ztile_ok(int t, size_t esize) { (void)esize; return t >= 0 && t < ZTILE_COUNT; }

inline int ztile_x(int t) {
  return (t == ZTILE_64x4 || t == ZTILE_64x8) ? 64 : ((t == ZTILE_32x8 || t == ZTILE_32x16) ? 32 : 16);
}
inline int ztile_y(int t) { return t == ZTILE_64x4 ? 4 : ((t == ZTILE_16x16 || t == ZTILE_32x16) ? 16 : 8); }

// Stage workspace: WS_COUNT arrays of `stride` elements back to back, so a
// kernel needs one base pointer for all of them (array pointers held in
// scalar registers would otherwise spill).
// With T_QUENCH six more follow: the quenched stress components, in the
// order of TauC; with T_ORDER2 also those and two more: the per-cell flags
// of the second-order switch (RG_*) and the second-order div u.
enum WsArr : int { WS_NUS = 0, WS_D, WS_UZ, WS_LNT, WS_Q0, WS_P0 = WS_Q0 + QOUT_COUNT,
                   WS_DIVB = WS_P0 + POUT_COUNT, WS_COUNT, WS_TQ0 = WS_COUNT,
                   WS_COUNT_QUENCH = WS_TQ0 + 6, WS_RGH = WS_COUNT_QUENCH, WS_D2,
                   WS_COUNT_ALL };

// Viscous stress components (eq. itv) and where they live: tau_xz on the
// y-edge, tau_yz on the x-edge, tau_zz, tau_xx, tau_yy at the centre, tau_xy
// on the z-edge.  Under quenching the passes' stress-only launches write
// the raw components to workspace arrays q(TauC) (pass Q's outputs, not
// yet written then), and the quench pass the quenched ones to WS_TQ0 + TauC.
enum TauC : int { TAU_XZ = 0, TAU_YZ, TAU_ZZ, TAU_XY, TAU_XX, TAU_YY, TAU_COUNT };

template <class T> struct ZWork {
  T* base;
  long long stride;
  T* lnpav;               // ln P_aver per plane of every box (BoxDev::poff; eq. pressure)
  // quenched stress (component c at tq + c * stride), or null: the passes
  // then form the stress themselves
  const T* tq = nullptr;
  // the second-order switch's flags, or null: sixth-order strain everywhere
  const T* rgh = nullptr;
  __host__ __device__ T* arr(int a) const { return base + (long long)a * stride; }
  __host__ __device__ T* q(int i) const { return arr(WS_Q0 + i); }
  __host__ __device__ T* pq(int i) const { return arr(WS_P0 + i); }
};

// Slices of a plane summed by separate workgroups for the plane means.
constexpr int kPlaneSlices = 8;

// Item queues of the persistent mode: 8 counters per launch, at most 9 launches.
constexpr int kQueueInts = 72;

struct ZLaunch {
  const BoxDev* boxes;
  const ZItem* items;     // device
  int nitems;
  int tile;               // ZTile of these items
  const ZItem* fitems;    // device: the work items of pass F, of tile ftile
  int nfitems;
  int ftile;
  int* queue;             // device, kQueueInts counters (persistent mode)
  int persistent;         // 0: one workgroup per item; 1: item queues
  int ncu;                // compute units of the device
  int nbox, nplanes;      // boxes; z planes of all boxes
  int stretched;          // some box has a stretched z axis (pass F's STR instantiation)
  hipStream_t stream;
  void (*mark)(void*, int);
  void* mark_ctx;
  void at(int pass) const { if (mark) mark(mark_ctx, pass); }
};

enum : int { DU_READ = 1, DU_WRITE = 2 };

template <class T> struct ZStageArgs {
  CP8<T> f;               // stage input state (ghosts filled)
  ZWork<T> w;
  Phys<T> ph;
  P8<T> du;               // the 2N-storage derivative (or dfdt when f_out is null)
  int du_mode;            // DU_READ: U = alpha dU + F;  DU_WRITE: store U
  P8<T> f_out;            // p[0] == nullptr: write F into du
  T alpha;
  double beta;            // the stage's beta; f_out = f + beta * dt * U
  double* dt_dev;         // device dt (nullptr: use dt_host)
  double dt_host;
  CPart* cpart;           // non-null: also compute the Courant dt into dt_dev
  const T* ztab;          // z-coefficient tables of wall boxes (BoxDev::zoff)
  T* lnavg;               // per plane of every box (BoxDev::poff): ln <e_m> (T_EDIFFAV)
  double* lnpart;         // kPlaneSlices partial sums per plane (T_EDIFFAV)
  double Cdt, Cdtd, nuB, eta_const;
};

template <class T> void launch_zstage(const ZLaunch& L, const ZStageArgs<T>& a);

// Pass F (mhd_zfinal.hip) in its tile shape L.ftile.
template <class T, bool PERS> void launch_final(const ZLaunch& L, const ZStageArgs<T>& a, int* q);
// Workgroups of a kernel that fit on the device at once (cached per kernel).
int zresident_groups(const void* kern, int block, int ncu);

// mhd_reductions: passes A1 and A2 in their reduction instantiations over
// the work items of L (grid mode), then the fold of the per-item partials
// red[L.nitems] into *tot.
template <class T>
void launch_zreduce(const ZLaunch& L, CP8<T> f, CP8<T> dfdt, const ZWork<T>& w, const Phys<T>& ph,
                    const T* ztab, RedItem* red, RedTotal* tot, double Cdt, double Cdtd, double Cdtr,
                    double nuB, double eta_const);

}  // namespace smhd
