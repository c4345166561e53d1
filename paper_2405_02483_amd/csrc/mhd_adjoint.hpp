// Discrete adjoint of the right-hand side: the RHS recorded once, on the host,
// as a straight-line program of whole-box operations (staggered stencils,
// max/mean over three cells, pointwise arithmetic) in the order of the
// equations of Sections 3-6 of the paper.  Running it forward keeps every
// intermediate in its own slot; running it backward applies each
// operation's transpose.  On a periodic axis the transpose of an
// interpolation is the interpolation of the opposite stagger, and the
// transpose of a derivative is minus the derivative of the opposite
// stagger; near the ends of a wall-bounded z axis, and on every plane of a
// stretched one, the z operators and their transposes use the box's
// coefficient tables (reduced orders, the end copy, the plane's Jacobian).
// The ghost fill of a wall box is not part of the program: its transpose
// is applied between the stages (vm_fill_vjp).
#pragma once

#include <vector>

#include "../../include/mhd.h"
#include "mhd_common.hpp"

namespace smhd {

enum VOp : int {
  V_STEN = 0,   // out = S(a): axis ax, family fam (0 interp, 1 deriv, 2 second-order
                //   deriv), form (0 dn, 1 up)
  V_ADD,        // out = a + b
  V_SUB,        // out = a - b
  V_MUL,        // out = a * b
  V_DIV,        // out = a / b
  V_SCALE,      // out = (k * geo) * a
  V_DIVC,       // out = a / k
  V_SQRT,       // out = sqrt(a)              (derivative 0 where out = 0)
  V_LOG,        // out = ln(a)
  V_EXP,        // out = exp(a)
  V_RELU,       // out = max(0, a)            (derivative 0 at a <= 0)
  V_FLOOR,      // out = a > k ? a : k        (derivative 0 at a <= k)
  V_NORM3,      // out = |(a, b, c)|          (derivative 0 at the origin)
  V_MAX3,       // out = max over cells i-1, i, i+1 along ax (first maximal one;
                //   the available ones at the ends of a wall-bounded z axis)
  V_MEAN3,      // out = (f[i-1] + f[i] + f[i+1]) / 3 along ax (the mean of the
                //   available ones at the ends of a wall-bounded z axis)
  V_FILL,       // out = k * geo (or k / h with G_HINV)
  V_ABS,        // out = |a|                  (derivative 0 at a = 0)
  V_D2,         // out = a[i+1] - 2 a[i] + a[i-1] along ax (0 on the end
                //   planes of a wall-bounded z axis)
  V_SDIV,       // out = b > 0 ? a / b : 0
  V_CAP,        // out = a < k ? a : k        (derivative 0 at a >= k)
  V_ROUGH,      // out = 1 if a cell touching position ax (0 centre, 1 x-, 2 y-,
                //   3 z-edge) has a second difference of a (ln rho) or b (ln e_m)
                //   above k, else 0 (a mask: no derivative)
  V_SEL,        // out = c > 1/2 ? b : a
  V_PMEAN,      // out = the mean of a over its z plane (of its box), at every
                //   cell of the plane (symmetric: its own transpose)
  V_COUNT
};

// Geometric factors multiplying the constant k of V_SCALE / V_FILL: the
// viscosity length factors of eq. nuij (BoxDev::lv, le), the energy
// diffusion's z length on the z-faces, the shock and Smagorinsky length,
// the box's smallest spacing and its reciprocal.  On a stretched z axis
// the z-dependent ones are the plane's (the per-plane table, ZJ_*).
enum VGeo : int { G_ONE = 0, G_LX, G_LY, G_LZ, G_H, G_HINV, G_LXY, G_LXZ, G_LYZ, G_LZF, G_HMIN };

// Axes of V_STEN / V_MAX3 / V_MEAN3 / V_D2.
enum VAxis : int { VX = 0, VY = 1, VZ = 2 };

struct VInstr {
  int op, out, a, b, c;
  int ax, fam, form, geo, pad;
  double k;
};

// Slots 0..7 hold the state (rho, px, py, pz, e, bx, by, bz); out[v] is the
// slot of the time derivative of variable v.
struct VProgram {
  std::vector<VInstr> code;
  int nslots = 8;
  int out[8];
};

// dt: the step's (the div B diffusion's coefficient); 0 leaves that term out
VProgram build_rhs_program(const mhd_params& p, double dt = 0.0);

// A program with storage assigned.  Forward values that no transpose reads
// share slots once their last reader has run; cotangents are allocated over
// their live range in the reverse sweep, and the first contribution to a
// cotangent overwrites it (no clearing pass).
struct VStep {
  VInstr f;                  // forward instruction on value slots
  int cout, ca, cb, cc;      // cotangent slots of out, a, b, c (-1: none)
  int over;                  // bit 0/1/2: the contribution to ca/cb/cc overwrites
};

// The forward run in groups, one launch each: a group starts with any
// operation (the only one that may read neighbouring cells) and continues
// with pointwise operations, up to kGroupMax.  Results made inside a group
// pass through a per-thread register file in LDS and are stored to their
// value slot only when a later group or a transpose reads them.
constexpr int kGroupMax = 16;
constexpr int kBGroupMax = 32;   // transposes per launch of the reverse sweep

struct VFused {
  VInstr f;                  // value slots (f.out: -1 if the result is not stored)
  int la, lb, lc;            // register of each operand made in this group (-1: memory)
  int pad;
};

struct VGroup { int first, count; };

struct VPlan {
  std::vector<VStep> steps;  // per operation: value slots of what the transposes read
  std::vector<VFused> fused; // the same operations for the grouped forward run
  std::vector<VGroup> groups;
  // the reverse sweep in groups, one launch each: bsteps holds the steps in
  // execution order (last operation first); a group starts with any
  // transpose (the only one that may read neighbouring cells' cotangents)
  // and continues with pointwise transposes
  std::vector<VStep> bsteps;
  std::vector<VGroup> bgroups;
  int nval = 0;              // value slots (0..7: the state)
  int ncot = 0;              // cotangent slots
  int cout[8];               // cotangent slot seeded with each output's cotangent
  int cin[8];                // cotangent slot of each input (-1: the input is unused)
};

VPlan plan_program(const VProgram& prog);

struct VLaunch {
  const BoxDev* boxes;
  const Blk* tab;
  int nblk;
  hipStream_t stream;
  int nbox, nplanes;      // boxes; z planes of all boxes (BoxDev::poff)
  double* pm;             // nplanes values: plane means (V_PMEAN)
  const void* ztab;       // z-coefficient tables of wall boxes (BoxDev::zoff), compute type
  const Blk* gtab;        // blocks over the ghost planes of wall boxes
  int nghost_blk;
};

// Forward: value slots base + s * stride (slots 0..7 filled by the caller);
// d_fused is plan.fused in device memory.
// Backward: cotangent slots cbase + s * stride, with the outputs' slots
// (plan.cout) seeded by the caller; afterwards slot plan.cin[v] holds
// (dF/df_v)^T of the seed.  d_bsteps is plan.bsteps in device memory.
template <class T>
void vm_forward(const VLaunch& L, const VPlan& plan, const VFused* d_fused, T* base, long long stride);
template <class T>
void vm_backward(const VLaunch& L, const VPlan& plan, const VStep* d_bsteps, const T* base, T* cbase,
                 long long stride);

// y[v] = a * y[v] + b * x[v] for the 8 fields (x may be null: y = a * y).
template <class T> void vm_axpby8(const VLaunch& L, P8<T> y, CP8<T> x, double a, double b);

// Closed walls (Section 10): the transpose of the ghost fill at the filled
// state s, in place: g holds the cotangent of the filled state on entry and
// that of the state before the fill on exit (zero in the ghost planes and on
// the two wall faces of p_z, which the fill overwrites).  tmp: 6 arrays of
// the packed field size (only their ghost cells are used).
template <class T> void vm_fill_vjp(const VLaunch& L, CP8<T> s, P8<T> g, T* tmp, long long stride);
// Closed walls: zero a cotangent of the right-hand side where the
// right-hand side itself is zeroed (ghost planes; p_z on the wall faces).
template <class T> void vm_wall_mask(const VLaunch& L, P8<T> g);

}  // namespace smhd
