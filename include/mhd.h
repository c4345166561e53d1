/*
 * mhd.h - C ABI of libstaggermhd: the staggered-mesh compressible MHD
 * right-hand side and its low-storage third-order Runge-Kutta advance on
 * AMD Instinct MI355X (gfx950), after Stein, Nordlund, Collet & Trampedach,
 * "The Stagger Code for Accurate and Efficient, Radiation-Coupled MHD
 * Simulations" (arXiv:2405.02483).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * State.  Eight arrays, always in this order (Section 4.1 "Centering"):
 *     0 rho   density                        cell centre
 *     1 px    momentum density, x            x-face at the lower index side
 *     2 py    momentum density, y            y-face
 *     3 pz    momentum density, z            z-face
 *     4 e     internal energy per volume     cell centre   (eq. ien: rho*e)
 *     5 bx    magnetic field, x              x-face
 *     6 by    magnetic field, y              y-face
 *     7 bz    magnetic field, z              z-face
 *   Element (i, j, k) of box b sits at offset box_offset(b) + (k*ny + j)*nx + i
 *   (x fastest), k = 0 .. nz + 2*ngz - 1 counting ghost planes.  A face
 *   array's element i is the face between cells i-1 and i.
 *   Boxes of a context are packed back to back in the same eight arrays
 *   (ensembles); mhd_box_offset() gives each box's first element.
 * Memory.  Every field pointer is a DEVICE pointer to a caller-owned array of
 *   mhd_field_elems() elements of the context's dtype (float or double),
 *   at least 16-byte aligned.  The library never frees caller memory.  The
 *   context owns its own device workspace (intermediate arrays, reduction
 *   partials), allocated in mhd_init / on first use and freed by
 *   mhd_destroy.
 * Streams.  All calls enqueue work on the HIP stream given to mhd_init and
 *   return without waiting, except mhd_reductions, which waits for its own
 *   result.  Calls that share one context must not run concurrently.
 * Errors.  Every int-returning call returns MHD_OK (0) or a negative code and
 *   never aborts; mhd_last_error() describes the last failure of the context.
 *   Argument checks (null pointers, sizes, dtype) happen before any work is
 *   enqueued.
 */
#ifndef STAGGER_MHD_H
#define STAGGER_MHD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MHD_OK = 0,
    MHD_EINVAL = -1,        /* bad argument (null pointer, size, parameter)   */
    MHD_ENOMEM = -2,        /* device allocation failed                       */
    MHD_EHIP = -3,          /* a HIP runtime call failed                      */
    MHD_EDTYPE = -4,        /* unknown dtype                                  */
    MHD_ENONFINITE = -5,    /* non-finite or non-positive state detected      */
    MHD_EUNSUPPORTED = -6   /* valid request the library does not implement   */
};

enum { MHD_F32 = 0, MHD_F64 = 1 };

/* z boundary.  x and y are always periodic (Section 10). */
enum {
    MHD_BC_PERIODIC = 0,    /* periodic z, ngz must be 0                       */
    MHD_BC_WALL = 1         /* closed walls with ngz >= 5 ghost planes per side */
};

/* Term switches (a finer form of the &vars namelist switches do_density,
 * do_momenta, do_energy, do_mhd of the paper's appendix).                    */
#define MHD_T_CONT     (1u << 0)   /* eq. mass                                 */
#define MHD_T_ADV      (1u << 1)   /* -div(rho u u), -div(e u)                 */
#define MHD_T_PRES     (1u << 2)   /* -grad P, -P div u                        */
#define MHD_T_VISC     (1u << 3)   /* div tau (eq. itv), Q_visc (eq. vdiss)    */
#define MHD_T_LORENTZ  (1u << 4)   /* J x B                                    */
#define MHD_T_INDUCT   (1u << 5)   /* -u x B in E (eq. ohm)                    */
#define MHD_T_RESIST   (1u << 6)   /* eta J in E and Joule heating             */
#define MHD_T_EDIFF    (1u << 7)   /* energy diffusion (eq. ediffuse)          */
#define MHD_T_GRAV     (1u << 8)   /* constant gravity along -z (Table 1)      */
#define MHD_T_ALL      ((1u << 9) - 1u)
/* Newtonian heating/cooling (eq. NewtonCool, eq. rhocool): a source
 * -rho (e_m - e_cool) / t_cool in the equation for e (e_m = e / rho, the
 * energy per unit mass), times a density factor chosen by cool_cut.  Not
 * part of MHD_T_ALL.  The RK3 step is stable for dt < 2.5 t_cool; the
 * Courant dt does not include this limit.                                  */
#define MHD_T_COOL     (1u << 9)
/* Coriolis force -2 rho Omega x u (eq. mom), written -2 Omega x p with each
 * momentum component interpolated to the face of the one it drives.  Not
 * part of MHD_T_ALL.                                                        */
#define MHD_T_CORI     (1u << 10)
/* With MHD_T_EDIFF: energy diffusion of the fluctuations about the
 * horizontal mean (eq. ediffav): the z flux differentiates
 * ln e_m - ln <e_m>, <e_m> the mean of e_m over each z plane of the box
 * (ghost planes included, as filled).  Not part of MHD_T_ALL.              */
#define MHD_T_EDIFFAV  (1u << 11)
/* With MHD_T_PRES: grad P in the momentum equation through
 * q = ln(P / P_aver), P_aver the mean of P over each z plane of the box
 * (eq. pressure): on a face f of axis a, exp(adn(ln P_aver)) exp(adn(q))
 * (ddadn(q) + ddadn(ln P_aver)).  Exact for an exponential atmosphere.  Not
 * part of MHD_T_ALL.                                                       */
#define MHD_T_LNP      (1u << 12)
/* div B diffusion: c_divb min(dx, dy, dz)^2 / dt grad(div B) added to the
 * rate of B, div B at cell centres from the up derivatives, its gradient on
 * the faces from the down derivatives.  It needs the step's dt, so
 * mhd_step and mhd_step_adjoint include it, mhd_rhs and mhd_rhs_adjoint
 * (no dt) leave it out.  Not part of MHD_T_ALL.                            */
#define MHD_T_DIVB     (1u << 13)
/* Smagorinsky viscosity (eq. nusmag): the rate nu_S = c_smag [2(sum_i S_ii^2
 * - (div u)^2/3 + sum_{i!=j} S_ij^2)]^(1/2), off-diagonal strain
 * interpolated to the cell centre, added to the Richtmyer-Morton viscosity
 * as the speed h_min nu_S before the maximum and mean, so that
 * nu_ii = dx_i h_min <nu_S> (eq. nuij2's (dx_i)^2 <nu> on cubic cells).
 * Ignored with nu_const > 0.  Not part of MHD_T_ALL.                       */
#define MHD_T_SMAG     (1u << 14)
/* Spread the viscosity by the maximum over five adjacent cells along each
 * axis instead of three (Section 6.1.1, &pde do_max5).  Not part of
 * MHD_T_ALL.                                                               */
#define MHD_T_MAX5     (1u << 15)
/* Quenching of the viscous stress (Section 6.2, eq. quench): each of the six
 * components tau is multiplied by min(max of q over the 3x3x3 neighbourhood,
 * q_lim), q = D2 / (|tau| + D2 / q_max), with D2 the sum over the three axes
 * of the absolute second differences of tau (none across the ends of a
 * wall-bounded axis; q = 0 where tau and D2 vanish).  The quenched stress
 * drives the momentum and the viscous heating.  Needs MHD_T_VISC to have
 * an effect.  Not part of MHD_T_ALL.                                        */
#define MHD_T_QUENCH   (1u << 16)
/* Second-order strain where the state is rough (Section 3, after eq. itv):
 * a cell is rough where some axis's absolute second difference of ln rho
 * or of ln e_m (e_m = e / rho) exceeds d2_lim (none across the ends of a
 * wall-bounded axis); a strain component of the viscous stress (and the
 * div u of its c1 term) takes the second-order staggered derivatives
 * wherever a cell touching its position is rough.  The viscous heating
 * uses the same strain.  Needs MHD_T_VISC to have an effect.  Not part of
 * MHD_T_ALL.                                                               */
#define MHD_T_ORDER2   (1u << 17)

/* One box of the mesh (&grid namelist: mx, my, mz, sx, sy, sz). */
typedef struct {
    int32_t nx, ny, nz;     /* interior cells; each >= 6                       */
    int32_t ngz;            /* ghost planes per z side: 0 periodic; walls: 5 <= ngz <= nz */
    int32_t bc_z;           /* MHD_BC_PERIODIC or MHD_BC_WALL                  */
    int32_t reserved;       /* must be 0                                       */
    double Lx, Ly, Lz;      /* box size; dx = Lx/nx, dy = Ly/ny, dz = Lz/nz    */
    /* Stretched z (Section 4.2; walls only), or NULL for uniform dz: host
     * array of the nz + 2 ngz cell-centre heights (ghost planes included),
     * finite and strictly increasing, copied by mhd_init (Lz is then
     * unused).  The grid interval dz/dxi is the derivative of the
     * not-a-knot cubic spline through (k, zc[k]), at the centres and the
     * faces; every z derivative is the index-space stencil times the
     * inverse interval at its output; nu_zz's length is the centre interval,
     * the x-/y-edge lengths max(dx or dy, face interval), the energy
     * diffusion's z length the face interval, the shock and Smagorinsky h
     * the cell's smallest spacing, cell volumes dx dy dz_c; the Courant,
     * div B diffusion and constant-viscosity h is the box's smallest
     * spacing.  MHD_EINVAL for a periodic box or a non-increasing zc.      */
    const double* zc;
} mhd_box;

/* Physical and numerical parameters (&pde, &run, &force namelists).         */
typedef struct {
    int32_t dtype;          /* MHD_F32 or MHD_F64: storage and arithmetic      */
    int32_t nbox;           /* number of boxes (>1: packed ensemble)           */
    const mhd_box* boxes;   /* host array of nbox boxes, copied by mhd_init    */
    double gamma;           /* ideal-gas ratio of specific heats, > 1          */
    double mu;              /* permeability; J = curl B / mu (eq. mom)         */
    double gz;              /* gravity along -z (with MHD_T_GRAV)              */
    double nu1, nu2, nu3;   /* eq. RMnu: c_v, c_sh, c_w                        */
    double nu_const;        /* > 0: constant viscosity, nu_ij = nu_const for
                               every component on any cell shape (Section 6.1) */
    double c1;              /* eq. itv                                         */
    double nuE;             /* eq. ediffuse: c_E                               */
    double nuB;             /* magnetic diffusivity = nuB * edge viscosity     */
    double eta_const;       /* > 0: constant magnetic diffusivity instead      */
    double Cdt, Cdtd, Cdtr; /* eq. courantcond                                 */
    uint32_t terms;         /* MHD_T_* bit set                                 */
    int32_t reserved;       /* must be 0                                       */
    /* with MHD_T_COOL (eq. NewtonCool, eq. rhocool); ignored otherwise:     */
    double e_cool;          /* target energy per unit mass, finite            */
    double t_cool;          /* time scale, > 0                                 */
    double rho_cool;        /* cut-off density, > 0 when cool_cut != 0         */
    int32_t cool_cut;       /* 0: factor 1; 1: r^2/(1+r^2) (weak cooling at low
                               density); 2: 1/(1+r^2) (at high); r = rho/rho_cool */
    int32_t reserved2;      /* must be 0                                       */
    double omega[3];        /* with MHD_T_CORI: rotation vector, finite        */
    double c_divb;          /* with MHD_T_DIVB: >= 0 and at most the RK3 limit
                               2.5127 / (K^2 h_min^2 sum_a 1/h_a^2), K = 2.48333
                               (0.1358 on cubic cells); MHD_EINVAL above it    */
    double c_smag;          /* with MHD_T_SMAG: the Smagorinsky constant, finite
                               and >= 0 (&pde Csmag, typically 0.1 - 0.15)     */
    double q_max, q_lim;    /* with MHD_T_QUENCH: eq. quench, both finite and
                               > 0 (&quench qmax = 8, qlim = 2)                */
    double d2_lim;          /* with MHD_T_ORDER2: the roughness limit, finite
                               (&pde d2lnr_lim = 0.3)                          */
} mhd_params;

/* Conserved totals and diagnostics over the interior cells (float64).     */
typedef struct {
    double mass;            /* sum rho dV                                      */
    double mom[3];          /* sum p_a dV                                      */
    double ekin;            /* sum over faces of p_a^2 / (2 rho_a) dV           */
    double emag;            /* sum over faces of B_a^2 / (2 mu) dV              */
    double eint;            /* sum e dV                                        */
    double divb_max;        /* max |div B| at centres                          */
    double divb_rms;        /* rms of div B                                    */
    double bmax;            /* max |B_a| over face components                  */
    double umax;            /* max |u_a| over face components                  */
    double cmax;            /* max (c_s + c_A + |u_perp B|) at centres         */
    double numax;           /* max diffusion speed max(nu, eta hmax/hmin), with
                               nu, eta the speed-like viscosity and resistivity */
    double ratemax;         /* max(|drho/dt|/rho, |d e_m/dt|/e_m); 0 if no dfdt */
    double dt;              /* eq. courantcond: min of the limits below        */
    double dt_wave, dt_diff, dt_rate;   /* each limit (dt_rate = inf if none)  */
    int64_t dt_argmax;      /* box-local flat index of the cell setting dt     */
    int32_t dt_box;         /* box of that cell                                */
    int32_t dt_limit;       /* 0 wave, 1 diffusion, 2 rate                     */
    int64_t n_nonfinite;    /* non-finite values among the 8 fields            */
    int64_t n_nonpositive;  /* cells with rho <= 0 or e <= 0                    */
} mhd_stats;

typedef struct mhd_ctx mhd_ctx;

/* Create a context for the boxes and parameters in *p, bound to hip_stream
 * (a hipStream_t; NULL = the null stream) on the current device.  Checks
 * every box (n >= 6; walls need ngz >= 5 and ngz == 0 otherwise; fewer
 * than 2^31 cells per box, ghost planes included) and
 * parameter (gamma > 1, mu > 0, viscosity and diffusion coefficients >= 0)
 * and allocates the workspace.  On success *out owns it.                   */
int mhd_init(const mhd_params* p, void* hip_stream, mhd_ctx** out);

/* Release the context and its workspace (waits for the stream).  NULL ok.  */
void mhd_destroy(mhd_ctx* ctx);

/* Text of the last error of ctx (or of the last failed mhd_init if NULL).  */
const char* mhd_last_error(const mhd_ctx* ctx);

/* Elements per field array (all boxes, ghost planes included).             */
int64_t mhd_field_elems(const mhd_ctx* ctx);

/* First element of box b in the packed arrays; -1 if b is out of range.    */
int64_t mhd_box_offset(const mhd_ctx* ctx, int32_t b);

/* dfdt = F(f): the time derivatives of the eight variables (eqs. mass, mom,
 * ien, indu, ohm, itv, vdiss, RMnu, nuij, ediffuse).  With walls the ghost
 * planes of f are filled first (written in place; interior untouched) and
 * dfdt is zero in ghost planes and for pz on the wall faces (Section 10).
 * f and dfdt must not overlap.                                             */
int mhd_rhs(mhd_ctx* ctx, void* const f[8], void* const dfdt[8]);

/* mhd_rhs for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * result is that of mhd_rhs, bit for bit (same kernels, same order).  The
 * call allocates nothing: its per-call scratch (stage workspace, per-plane
 * tables, queue counters) lives in a static device array of 64 MiB that
 * each GPU holds from the first mhd_init on it until the process ends; the
 * context's tables come from mhd_init.  That fits about 490,000 cells of
 * float32 or 245,000 of float64 (ghost planes included; 34 arrays per cell,
 * 40 with MHD_T_QUENCH, 42 with MHD_T_ORDER2, plus small per-plane
 * tables).  MHD_EINVAL, with the bytes needed in
 * mhd_last_error, when the context's boxes need more; MHD_EHIP when the array is
 * not available on the device.  Every call on one GPU shares the one array
 * and overwrites its contents: calls that overlap on one GPU (other
 * streams, other contexts, other threads) race and must be ordered by the
 * caller.                                                                  */
int mhd_rhs_noalloc(mhd_ctx* ctx, void* const f[8], void* const dfdt[8]);

/* Advance f by nsteps steps of the low-storage RK3 scheme (eqs. ddt,
 * tupdate, tconst):  per stage i, dU <- alpha_i dU + F(f),
 * f <- f + beta_i dt dU.  dt > 0: that fixed step.  dt == 0: every step
 * uses the Courant step (eq. courantcond, wave and diffusion limits) of its
 * own initial state, computed on the device during the first stage; read
 * the last one with mhd_last_dt.  The result is in f.  tmp1, tmp2 (8 arrays
 * each) hold the stage states, dU the 2N-storage derivative; their contents
 * on return are unspecified.  With walls, ghost planes are refilled before
 * every evaluation of F and after the last stage.                          */
int mhd_step(mhd_ctx* ctx, void* const f[8], void* const tmp1[8],
             void* const tmp2[8], void* const dU[8], double dt, int32_t nsteps);

/* Discrete adjoint of one mhd_step at fixed dt (dt is not differentiated):
 * gbar_out = (d f_{n+1} / d f_n)^T gbar_in, evaluated at the state f_n.
 * Non-smooth points use: max over three cells routes to the first maximal
 * cell (order i-1, i, i+1; passes along x, then y, then z); max(0, x), |v|
 * and the viscosity floor have zero derivative on their flat side.  Every
 * term bit is differentiated, the plane means of MHD_T_EDIFFAV and
 * MHD_T_LNP included (each mean depends on every cell of its plane).  With
 * closed walls the step's ghost fills (before every evaluation of F and
 * after the last stage) and the zeroing of F in the ghost planes and on the
 * wall faces are transposed too, so gbar_out is zero in the ghost planes
 * and for p_z on the wall faces (values the step overwrites).  On a
 * stretched z axis the per-plane Jacobians and lengths are constants of
 * the differentiation, as dx, dy are.  dt must be finite and
 * > 0 (MHD_EINVAL otherwise: the Courant step of mhd_step's dt == 0 is not
 * differentiated).  f_n is not modified; gbar_in and gbar_out must not
 * overlap.                                                                 */
int mhd_step_adjoint(mhd_ctx* ctx, void* const f_n[8], double dt,
                     void* const gbar_in[8], void* const gbar_out[8]);

/* Discrete adjoint of mhd_rhs: fbar = (dF/df)^T wbar at the state f (the
 * same non-smooth conventions as mhd_step_adjoint).  With walls F is what
 * mhd_rhs computes from f, ghost fill included, and fbar is zero where the
 * fill overwrites f.  f and wbar are not modified; fbar must not overlap
 * them.  Allocates the adjoint workspace on first use.                     */
int mhd_rhs_adjoint(mhd_ctx* ctx, void* const f[8], void* const wbar[8],
                    void* const fbar[8]);

/* Float64 totals, diagnostics and the Courant time step (eq. courantcond)
 * of state f over the interior of all boxes; writes *out (host memory) and
 * waits for the stream.  dfdt may be NULL; if given (the time derivatives of
 * f) the rate limit Cdtr enters dt.  With walls, ghost planes of f are
 * filled first.  Returns MHD_ENONFINITE (after filling *out) when a
 * non-finite value or a non-positive rho or e is present.                  */
int mhd_reductions(mhd_ctx* ctx, void* const f[8], void* const dfdt[8],
                   mhd_stats* out);

/* div B cleaning in Fourier space (Section 3, eq. clean1, eq. clean2):
 * projects the magnetic field f[5..7] of every box in place onto its
 * discretely solenoidal part.  The potential phi solves ddxup(ddxdn(phi))
 * + ddyup(ddydn(phi)) + ddzup(ddzdn(phi)) = div B (div B from the up
 * derivatives at the centres), whose Fourier symbol is -(K_x^2 + K_y^2 +
 * K_z^2) with K the sixth-order derivative symbol (the mean mode's phi is
 * 0); then B_a -= ddadn(phi).  Afterwards the discrete div B is zero to
 * rounding; a discrete curl is unchanged; the other fields are untouched.
 * The projection is orthogonal for the sum of squares over the faces (the
 * down derivative is minus the transpose of the up one), so it is its own
 * adjoint.
 * Needs periodic boxes (MHD_EUNSUPPORTED with walls).  The first call
 * makes rocFFT plans per box shape and allocates scratch for the largest
 * box (about 3 of its fields), kept until mhd_destroy (MHD_ENOMEM,
 * MHD_EHIP on failure).  Returns without waiting.                          */
int mhd_divb_clean(mhd_ctx* ctx, void* const f[8]);

/* The dt of the last step taken with dt == 0 (waits for the stream).      */
int mhd_last_dt(mhd_ctx* ctx, double* dt);

/* Tile shape of the stage kernels: columns per workgroup, 0: 64x4,
 * 1: 32x8, 2: 16x16, 3: 16x8 (256 threads), 4: 64x8, 5: 32x16 (512
 * threads).  Any shape gives the same results (bit for bit); the default is
 * 32x8 (float32) or 16x8 (float64).  Other values: MHD_EINVAL.  Also sets
 * pass F to this shape (mhd_set_final_tile).                               */
int mhd_set_tile(mhd_ctx* ctx, int32_t tile);

/* Tile shape (as mhd_set_tile) and launch mode of the stage kernels.
 * persistent = 0: one workgroup per work item (box, column tile, z range).
 * persistent = 1: about one resident wave of workgroups, each taking work
 * items from a queue per XCD and from the other XCDs' queues once its own is
 * empty (load balance for ensembles of uneven boxes).  Results are the same
 * bit for bit in every tile shape and mode.  MHD_EINVAL on other values.   */
int mhd_set_launch(mhd_ctx* ctx, int32_t tile, int32_t persistent);

/* Current tile shape and launch mode.                                      */
int mhd_get_launch(const mhd_ctx* ctx, int32_t* tile, int32_t* persistent);

/* Tile shape of pass F alone (the divergences and the RK stage update), as
 * mhd_set_tile; mhd_set_tile and mhd_set_launch set it to their own shape.
 * Results are the same bit for bit.  MHD_EINVAL on other values.            */
int mhd_set_final_tile(mhd_ctx* ctx, int32_t tile);
int mhd_get_final_tile(const mhd_ctx* ctx, int32_t* tile);


/* Autotuner: times reps RK stages of the kind a step repeats (the right-hand
 * side of f with the stage update: dU read and written, the next state
 * written to scratch; after one mhd_rhs(f, dfdt) as warm-up) in every tile
 * shape and launch mode, in three rounds over all of them, keeps the
 * fastest (each candidate's best round) and, if ms is not NULL, writes the
 * milliseconds per stage to ms[2 * tile + persistent] (12 entries; 0 for a
 * shape not built for the context's dtype).  Then, with that shape for the
 * other passes, times every shape for pass F alone in both modes (three
 * rounds again), and keeps the fastest combination if it beats the uniform
 * launch by more than 1 % (mhd_get_launch, mhd_get_final_tile).  dfdt is
 * overwritten; with walls the ghost planes of f are filled.  Allocates 8
 * fields of scratch for the call (MHD_ENOMEM).  Waits for the stream.      */
int mhd_autotune(mhd_ctx* ctx, void* const f[8], void* const dfdt[8], int32_t reps,
                 double* ms);

/* Timing of the library's own kernel passes, for performance measurement.
 * Pass ids (index into the arrays of mhd_profile_read):                    */
enum {
    MHD_PASS_PRIM = 0,      /* A1: u_z, div u, speed-like viscosity            */
    MHD_PASS_NUS = 1,       /* (unused)                                        */
    MHD_PASS_MAX3 = 2,      /* (unused)                                        */
    MHD_PASS_MEAN3 = 3,     /* A2: max over three cells, three-cell mean, log  */
    MHD_PASS_EDGES = 4,     /* Q (two launches): x/y-edge quantities; Hz, Gzz  */
    MHD_PASS_CF = 5,        /* P: z-edge quantities, centre stresses, Hx, Hy   */
    MHD_PASS_FINAL = 6,     /* F (three launches): divergences, RK update      */
    MHD_PASS_GHOST = 7,     /* closed-wall ghost zones                          */
    MHD_PASS_REDUCE = 8,    /* float64 reductions incl. their viscosity chain   */
    MHD_PASS_ADJOINT = 9,   /* adjoint kernels                                  */
    MHD_PASS_COUNT = 10
};

/* enable != 0: from now on record a HIP event on the context's stream
 * before every kernel pass and after the last pass of each call; enable ==
 * 0: stop.  Either way the accumulated totals are reset.  Recording adds a
 * few microseconds per pass.                                               */
int mhd_profile(mhd_ctx* ctx, int32_t enable);

/* Waits for the stream, then writes for each pass q < n the accumulated GPU
 * milliseconds ms[q] (event to event on the context's stream) and the number
 * of timed launches count[q] since the last mhd_profile call.             */
int mhd_profile_read(mhd_ctx* ctx, double* ms, int64_t* count, int32_t n);

#ifdef __cplusplus
}
#endif

#endif /* STAGGER_MHD_H */
