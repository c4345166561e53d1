// Host-visible declarations shared by the kernel files and the C ABI layer.
#pragma once

#include "mhd_common.hpp"

namespace smhd {

// Physical parameters in the arithmetic type of the kernels.
template <class T> struct Phys {
  T gamma, gamma1, mu, inv_mu, gz;
  T nu1, nu2, nu3, nu_const, c1, nuE, nuB, eta_const;
  T e_cool, inv_tcool, inv_rho_cool;   // Newtonian cooling (with T_COOL)
  int cool_cut;
  T cor2[3];                            // 2 Omega (Coriolis force, with T_CORI)
  T c_divb;                             // div B diffusion coefficient (with T_DIVB)
  T c_smag;                             // Smagorinsky constant (with T_SMAG)
  T q_max, q_lim;                       // quenching (with T_QUENCH)
  T d2_lim;                             // roughness limit (with T_ORDER2)
  unsigned terms;
};

// Kernel passes, as reported by the timing hook (order = mhd.h MHD_PASS_*).
enum Pass : int {
  PASS_PRIM = 0, PASS_NUS, PASS_MAX3, PASS_MEAN3, PASS_EDGES, PASS_CF, PASS_FINAL,
  PASS_GHOST, PASS_REDUCE, PASS_ADJOINT, PASS_COUNT, PASS_END = -1
};

// Launch geometry shared by all cell kernels of a context.
struct Launch {
  const BoxDev* boxes;    // device
  const Blk* tab;         // device, nblk entries covering every cell
  int nblk;
  const Blk* gtab;        // device, blocks over the ghost planes of wall boxes
  int nghost_blk;
  hipStream_t stream;
  // optional timing hook: mark(mark_ctx, pass) before a pass starts and
  // mark(mark_ctx, PASS_END) after the last one of a sequence
  void (*mark)(void*, int);
  void* mark_ctx;
  void at(int pass) const { if (mark) mark(mark_ctx, pass); }
};

template <class T> void launch_ghost(const Launch& L, P8<T> f);

}  // namespace smhd
