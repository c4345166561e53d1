// Host-side view of the z-marching stage kernels (mhd_zmarch.hip).
#pragma once

#include "mhd_zmarch.hpp"

namespace smhd {

// Outputs of pass Q, in workspace order.
enum QOut : int {
  QOUT_GXZ = 0, QOUT_GZX, QOUT_EY, QOUT_LXY, QOUT_LZY, QOUT_QY,
  QOUT_GYZ, QOUT_GZY, QOUT_EX, QOUT_LYX, QOUT_LZX, QOUT_QX,
  QOUT_HZ, QOUT_GZZ, QOUT_CZZ, QOUT_COUNT
};

template <class T> struct QP { T* p[QOUT_COUNT]; };
template <class T> struct CQP { const T* p[QOUT_COUNT]; };

// Tile shapes (columns per workgroup, x by y) the stage kernels are built for.
enum ZTile : int { ZTILE_64x4 = 0, ZTILE_32x8 = 1, ZTILE_16x16 = 2, ZTILE_16x8 = 3, ZTILE_COUNT };

// Whether a tile shape is built for an element size (the 64x4 float64
// variant of pass F would exceed the 160 KB of LDS of a workgroup).
inline bool ztile_ok(int t, size_t esize) { return t >= 0 && t < ZTILE_COUNT && !(t == ZTILE_64x4 && esize == 8); }

inline int ztile_x(int t) { return t == ZTILE_64x4 ? 64 : (t == ZTILE_32x8 ? 32 : 16); }
inline int ztile_y(int t) { return t == ZTILE_64x4 ? 4 : (t == ZTILE_32x8 ? 8 : (t == ZTILE_16x16 ? 16 : 8)); }

template <class T> struct ZWork {
  T *nus, *D, *uz, *lnt;
  T* q[QOUT_COUNT];
};

struct ZLaunch {
  const BoxDev* boxes;
  const ZItem* items;     // device
  int nitems;
  int tile;               // ZTile of these items
  hipStream_t stream;
  void (*mark)(void*, int);
  void* mark_ctx;
  void at(int pass) const { if (mark) mark(mark_ctx, pass); }
};

template <class T> struct ZStageArgs {
  CP8<T> f;               // stage input state (ghosts filled)
  ZWork<T> w;
  Phys<T> ph;
  CP8<T> du_in;           // p[0] == nullptr: first stage
  P8<T> du_out;           // p[0] == nullptr: do not store dU
  P8<T> f_out;            // p[0] == nullptr: write F into du_out
  T alpha;
  double beta;            // the stage's beta; f_out = f + beta * dt * U
  double* dt_dev;         // device dt (nullptr: use dt_host)
  double dt_host;
  CPart* cpart;           // non-null: also compute the Courant dt into dt_dev
  double Cdt, Cdtd, nuB, eta_const;
};

template <class T> void launch_zstage(const ZLaunch& L, const ZStageArgs<T>& a);

}  // namespace smhd
