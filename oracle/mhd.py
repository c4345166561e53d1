"""Compressible MHD right-hand side on the staggered mesh, ghost-zone fill,
low-storage RK3 time step, Courant time step, conserved totals and the
discrete adjoint of one step.  Plain float64 CPU reference.

TEST INFRASTRUCTURE ONLY (see the package docstring).

State: a tuple of 8 float64 tensors ``[nzt, ny, nx]`` in the order
``rho, px, py, pz, e, bx, by, bz`` where ``e`` is the internal energy per
unit volume (rho times the energy per unit mass of eq. ien) and ``p`` the
momentum density.  ``nzt = nz + 2*ngz``; ``ngz = 0`` for a periodic z axis.

Readings of the paper taken here, where it is silent, ambiguous or
garbled:

* eq. mom, eq. itv: the viscous stress enters the momentum equation with the
  dissipative sign (+div tau with tau = +rho nu S), so that the viscous
  dissipation Q_visc of eq. vdiss is a heating term.
* eq. ohm: ``eta`` is a magnetic diffusivity, E = -u x B + eta curl B, and the
  Joule heating is eta |curl B|^2 / mu, which is eta J^2 with J = curl B/mu
  and resistivity mu*eta.
* eq. RMnu: the shock term is nu2 * h * max(0, -div u) (a length h = the
  smallest grid spacing turns the rate into a speed, and it acts only in
  compression); the viscosity is spread by a maximum over three cells and
  smoothed by a three-cell mean along x, then y, then z.
* eq. nuij: off-diagonal (edge) viscosities average ln(nu) and exponentiate.
* Constant viscosity (Section 6.1, nu_ij = const): every component nu_ij is
  nu_const on any cell shape; the smoothed speed-like viscosity is then
  nu_const / h_min, which sets the diffusive Courant limit.
* eq. ediffuse: the diffusive energy flux is nuE * rho * nu_ii * e_m *
  d(ln e_m)/dx_i with nu_ii = dx_i <nu>; the paper's extra factor dx_i would
  give the flux the wrong dimension and is dropped.
* Resistivity: eta = nuB * (edge viscosity), or a constant.
* Ideal-gas EOS: P = (gamma - 1) e.
* eq. NewtonCool: e there is the energy per unit mass, so the source in the
  equation for the energy per volume is Q = -rho (e_m - e_cool) / t_cool
  (e_m relaxes to e_cool on the time scale t_cool at fixed density), times
  one of the density cut-offs of eq. rhocool when one is chosen.
* eq. ediffav: <e>_horiz is the mean of the energy per unit mass over the
  x-y plane of each z level (ghost planes included, as filled), and the
  flux differentiates ln e_m - ln <e_m>_horiz; only the z component
  changes, since the plane mean does not vary along x or y.
* eq. pressure: P_aver is the mean of P over each z plane (ghost planes
  included, as filled); every component of grad P in the momentum equation
  takes the printed form exp(ln P_aver)_f exp(ln(P/P_aver))_f
  [d ln(P/P_aver) + d ln P_aver]_f with the staggered interpolation and
  derivative to the face f (the x and y derivatives of P_aver vanish).
* div B diffusion (the C_divb term of the induction equation): the printed
  term adds a scalar to a vector rate; it is read as the gradient of div B,
  C_divb min(dx, dy, dz)^2 / dt grad(div B), with div B at cell centres from
  the up derivatives and its gradient on the faces from the down
  derivatives.  It needs the step's dt, so only the RK step (or a right-hand
  side given dt) includes it.
* Section 6.1.1, maximum over three or five cells: with T_MAX5 the
  viscosity is spread by the maximum over five adjacent cells along each
  axis (the three-cell maximum applied twice), then smoothed by the
  three-cell mean as before.
* eq. nusmag, eq. nuij2 (Smagorinsky): nu_S = c_smag [2(sum_i S_ii^2 -
  (div u)^2/3 + sum_{i!=j} S_ij^2)]^(1/2), a rate, with the off-diagonal
  S_ij interpolated from its edge to the cell centre before squaring.  It
  enters the same chain as the Richtmyer-Morton viscosity as the speed
  h_min nu_S, added before the maximum and the mean (the paper combines the
  two "in varying proportions"), so that nu_ii = dx_i h_min <nu_S>: eq.
  nuij2's (dx_i)^2 <nu> on cubic cells.  The depth factor the paper applies
  "sometimes" in stratified runs is not used.
* eq. quench: the printed second line sets T to q_i times a bracket; read
  as the stress being multiplied by the bracket min(max(q_{i-1}, q_i,
  q_{i+1}), q_lim), which reduces smooth stress and raises a two-zone
  wiggle, as the text says.  In three dimensions Delta^2 T is the sum over
  the axes of the absolute second differences (absolute, so that q >= 0)
  and the maximum runs over the 3x3x3 neighbourhood, as for the viscosity.
  All six components are quenched, each at its own position, and the
  quenched stress enters both the momentum equation and the viscous
  heating (which keeps the total energy budget).
* Section 3 after eq. itv, the switch to second-order derivatives: read as
  the strain of the viscous stress (and the div u of its c1 term) taken
  with the second-order staggered derivative (the first pair of eq. deriv
  with weight 1) wherever a cell touching the component's position is
  rough: some axis's absolute second difference of ln rho or ln e_m
  (energy per unit mass, the paper's e) exceeds d2_lim (&pde d2lnr_lim =
  0.3).  The viscous heating uses the same strain.  The indicator is a
  mask: it carries no derivative.
* eq. mom, Coriolis force: -2 rho Omega x u = -2 Omega x p, with each
  momentum component carried to the face of the component it drives by the
  staggered interpolations (e.g. p_z at an x-face is xdn(zup(p_z))).
* eq. clean1, eq. clean2 (div B cleaning): the potential solves the
  Poisson equation of the discrete operators themselves, sum_a
  ddaup(ddadn(phi)) = div B, in Fourier space (symbol -(K_x^2 + K_y^2 +
  K_z^2) with K the sixth-order derivative symbol; the mean mode's phi is
  0), so the cleaned field is discretely solenoidal; periodic boxes only.
* Section 4.2 (stretched z axis): the grid interval is the derivative of
  the not-a-knot cubic spline through the cell-centre heights against the
  plane index, taken at each derivative's output (centre or face); z
  derivatives are index-space stencils times its inverse, interpolations
  and the ghost fill stay in index space, and every length factor takes
  the spacing at its own height (see viscosity_lengths, z_face_length).
"""
from dataclasses import dataclass, field, replace
import math

import torch

from .stagger import Ops, AX_X, AX_Y, AX_Z, DERIV6

__all__ = [
    "T_CONT", "T_ADV", "T_PRES", "T_VISC", "T_LORENTZ", "T_INDUCT",
    "T_RESIST", "T_EDIFF", "T_GRAV", "T_ALL", "T_HD", "T_IDEAL", "T_COOL", "T_CORI",
    "T_EDIFFAV", "T_LNP", "T_DIVB", "T_SMAG", "T_MAX5", "T_QUENCH", "T_ORDER2",
    "ALPHA", "BETA", "Grid", "Params", "ghost_fill", "rhs", "rhs_nofill",
    "step", "rk3", "courant", "stats", "step_vjp", "rhs_vjp", "FIELDS",
    "interior_slices", "smoothed_viscosity", "newton_cooling", "coriolis",
    "horizontal_ln_mean", "pressure_gradient_ln", "viscosity_lengths",
    "edge_viscosity", "smagorinsky_rate", "quench_factor", "rough_cells", "strain",
    "derivative_symbol", "divb_clean", "zgrid_intervals", "z_face_length",
]

FIELDS = ("rho", "px", "py", "pz", "e", "bx", "by", "bz")

# Term switches (finer than, and implying, the &vars namelist switches
# do_density / do_momenta / do_energy / do_mhd of the paper's appendix).
T_CONT = 1 << 0      # eq. mass
T_ADV = 1 << 1       # advection: -div(rho u u) and -div(e u)
T_PRES = 1 << 2      # -grad P and -P div u
T_VISC = 1 << 3      # div tau (eq. itv) and Q_visc (eq. vdiss)
T_LORENTZ = 1 << 4   # J x B
T_INDUCT = 1 << 5    # ideal part of E (eq. ohm: -u x B)
T_RESIST = 1 << 6    # eta J in E and Joule heating
T_EDIFF = 1 << 7     # energy diffusion (eq. ediffuse)
T_GRAV = 1 << 8      # constant gravity along -z (Forcing, Table 1)
T_ALL = (1 << 9) - 1
T_COOL = 1 << 9      # Newtonian cooling (eq. NewtonCool); not part of T_ALL
T_CORI = 1 << 10     # Coriolis force (eq. mom); not part of T_ALL
T_EDIFFAV = 1 << 11  # with T_EDIFF: diffuse fluctuations about the plane mean (eq. ediffav)
T_LNP = 1 << 12      # with T_PRES: grad P through ln(P / P_aver) (eq. pressure)
T_DIVB = 1 << 13     # div B diffusion C_divb h^2 / dt grad(div B); needs the step's dt
T_SMAG = 1 << 14     # Smagorinsky viscosity added to the speed-like one (eq. nusmag)
T_MAX5 = 1 << 15     # spread the viscosity by the maximum over five cells (do_max5)
T_QUENCH = 1 << 16   # quench each viscous stress component (eq. quench)
T_ORDER2 = 1 << 17   # second-order strain where ln rho or ln e_m is rough (after eq. itv)
T_HD = T_CONT | T_ADV | T_PRES | T_VISC | T_EDIFF
T_IDEAL = T_CONT | T_ADV | T_PRES | T_LORENTZ | T_INDUCT

# eq. tconst (as printed, six digits)
ALPHA = (0.0, -0.641874, -1.31021)
BETA = (0.46173, 0.924087, 0.390614)

NU_FLOOR = 1e-30


def zgrid_intervals(zc):
    """Grid intervals dz/dxi of a stretched z axis (Section 4.2: the
    Jacobian is the inverse of the grid interval, from a spline fit, at the
    centre of each derivative).  zc: the heights of the n cell centres
    (xi = 0..n-1, strictly increasing).  The not-a-knot cubic spline through
    (k, zc[k]) has second derivatives M solving, with unit spacing,
    M[k-1] + 4 M[k] + M[k+1] = 6 (zc[k+1] - 2 zc[k] + zc[k-1]) for interior k
    and M[0] - 2 M[1] + M[2] = 0, M[n-3] - 2 M[n-2] + M[n-1] = 0 (a
    continuous third derivative at the second and the second-last knots).
    Returns (dzc, dzf): its derivative at the centres xi = k and at the
    faces xi = k - 1/2 (face 0 from the first interval's cubic)."""
    z = torch.as_tensor(zc, dtype=torch.float64)
    n = z.shape[0]
    if n < 4:
        raise ValueError("a stretched axis needs at least 4 planes")
    A = torch.zeros(n, n, dtype=torch.float64)
    r = torch.zeros(n, dtype=torch.float64)
    A[0, 0], A[0, 1], A[0, 2] = 1.0, -2.0, 1.0
    A[n - 1, n - 3], A[n - 1, n - 2], A[n - 1, n - 1] = 1.0, -2.0, 1.0
    for k in range(1, n - 1):
        A[k, k - 1], A[k, k], A[k, k + 1] = 1.0, 4.0, 1.0
        r[k] = 6.0 * (z[k + 1] - 2.0 * z[k] + z[k - 1])
    M = torch.linalg.solve(A, r)
    # on [k, k+1]: S(xi) = M_k (k+1-xi)^3/6 + M_{k+1} (xi-k)^3/6
    #                    + (z_k - M_k/6)(k+1-xi) + (z_{k+1} - M_{k+1}/6)(xi-k)
    def slope(k, t):      # S'(k + t) on the interval [k, k+1]
        return (-M[k] * (1.0 - t) ** 2 / 2.0 + M[k + 1] * t ** 2 / 2.0
                + (z[k + 1] - M[k + 1] / 6.0) - (z[k] - M[k] / 6.0))
    dzc = torch.stack([slope(k, 0.0) if k < n - 1 else slope(n - 2, 1.0) for k in range(n)])
    dzf = torch.stack([slope(k - 1, 0.5) if k > 0 else slope(0, -0.5) for k in range(n)])
    return dzc, dzf


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    ngz: int = 0          # ghost planes per z side (5 with walls)
    wall: bool = False    # z bounded by closed walls (else periodic)
    Lx: float = 1.0
    Ly: float = 1.0
    Lz: float = 1.0
    # stretched z (walls only): the heights of the nz + 2 ngz cell centres;
    # None: uniform, dz = Lz / nz
    zc: tuple = None

    @property
    def nzt(self):
        return self.nz + 2 * self.ngz

    @property
    def stretched(self):
        return self.zc is not None

    def zintervals(self):
        """(dzc, dzf) per plane (tensors of nzt), stretched or uniform."""
        if self.zc is None:
            d = torch.full((self.nzt,), self.dz, dtype=torch.float64)
            return d, d
        if not self.wall or len(self.zc) != self.nzt:
            raise ValueError("a stretched z axis needs walls and nz + 2 ngz heights")
        return zgrid_intervals(self.zc)

    @property
    def dx(self):
        return self.Lx / self.nx

    @property
    def dy(self):
        return self.Ly / self.ny

    @property
    def dz(self):
        return self.Lz / self.nz

    @property
    def hmin(self):
        if self.zc is not None:
            return min(self.dx, self.dy, float(self.zintervals()[0].min()))
        return min(self.dx, self.dy, self.dz)

    @property
    def hmax(self):
        if self.zc is not None:
            return max(self.dx, self.dy, float(self.zintervals()[0].max()))
        return max(self.dx, self.dy, self.dz)

    def ops(self):
        if self.zc is not None:
            dzc, dzf = self.zintervals()
            return Ops(self.dx, self.dy, self.dz, wall_z=self.wall, jz=(1.0 / dzc, 1.0 / dzf))
        return Ops(self.dx, self.dy, self.dz, wall_z=self.wall)


@dataclass(frozen=True)
class Params:
    gamma: float = 5.0 / 3.0
    mu: float = 1.0
    gz: float = 0.0           # gravity acceleration along -z
    nu1: float = 0.02         # c_v   (eq. RMnu)
    nu2: float = 1.0          # c_sh
    nu3: float = 0.02         # c_w
    nu_const: float = 0.0     # >0: constant viscosity nu_ij = nu_const
    c1: float = 0.0           # eq. itv
    nuE: float = 1.0          # eq. ediffuse
    nuB: float = 1.0          # eta = nuB * edge viscosity
    eta_const: float = 0.0    # >0: constant magnetic diffusivity
    Cdt: float = 0.3          # eq. courantcond
    Cdtd: float = 0.7
    Cdtr: float = 0.1
    terms: int = T_ALL
    e_cool: float = 0.0       # eq. NewtonCool: target energy per unit mass
    t_cool: float = 1.0       # its time scale
    rho_cool: float = 1.0     # eq. rhocool: cut-off density
    cool_cut: int = 0         # 0 none, 1 low-density cut-off, 2 high-density
    omega: tuple = (0.0, 0.0, 0.0)   # rotation vector of the Coriolis force
    c_divb: float = 0.0       # coefficient of the div B diffusion (< 0.11)
    c_smag: float = 0.0       # Smagorinsky constant (eq. nusmag; &pde Csmag)
    q_max: float = 8.0        # eq. quench, &quench qmax
    q_lim: float = 2.0        # eq. quench, &quench qlim
    d2_lim: float = 0.3       # second-order strain above this |D2 ln rho|, |D2 ln e_m| (&pde d2lnr_lim)


def interior_slices(grid):
    """z-plane ranges of the interior: (centred-in-z fields, z-face fields)."""
    if not grid.wall:
        return slice(0, grid.nzt), slice(0, grid.nzt)
    g0, g1 = grid.ngz, grid.ngz + grid.nz
    return slice(g0, g1), slice(g0, g1)


# ---------------------------------------------------------------------------
def _safe_norm3(a, b, c):
    """sqrt(a^2+b^2+c^2) with zero derivative where the vector vanishes."""
    s = a * a + b * b + c * c
    pos = s > 0
    return torch.where(pos, torch.sqrt(torch.where(pos, s, torch.ones_like(s))),
                       torch.zeros_like(s))


def _relu(x):
    """max(0, x); derivative 1 where x > 0 and 0 elsewhere."""
    return torch.where(x > 0, x, torch.zeros_like(x))


def smoothed_viscosity(f, grid, par, O=None):
    """The viscosity <nu>_{max smooth} at cell centres (Section 6.1.1).

    Returns (nu_tilde, pieces) where pieces holds the centred primitives the
    Courant condition reuses.
    """
    O = O or grid.ops()
    rho, px, py, pz, e, bx, by, bz = f
    h = grid.hmin
    if grid.stretched and not par.nu_const > 0:
        # the local smallest spacing of each plane's cells
        h = torch.clamp(grid.zintervals()[0], max=min(grid.dx, grid.dy)).view(-1, 1, 1)
    P = (par.gamma - 1.0) * e
    ux, uy, uz = px / O.xdn(rho), py / O.ydn(rho), pz / O.zdn(rho)
    ubx, uby, ubz = O.xup(ux), O.yup(uy), O.zup(uz)
    bbx, bby, bbz = O.xup(bx), O.yup(by), O.zup(bz)
    D = O.ddxup(ux) + O.ddyup(uy) + O.ddzup(uz)
    cs = torch.sqrt(par.gamma * P / rho)
    ca = _safe_norm3(bbx, bby, bbz) / torch.sqrt(par.mu * rho)
    if par.nu_const > 0:
        nus = torch.full_like(rho, par.nu_const / grid.hmin)
    else:
        nus = (par.nu1 * _safe_norm3(ubx, uby, ubz)
               + par.nu3 * (cs + ca)
               + par.nu2 * h * _relu(-D))
        if par.terms & T_SMAG:
            nus = nus + par.c_smag * h * smagorinsky_rate(ux, uy, uz, D, O)
    mx = O.max5 if par.terms & T_MAX5 else O.max3
    m = mx(mx(mx(nus, AX_X), AX_Y), AX_Z)
    nt = O.mean3(O.mean3(O.mean3(m, AX_X), AX_Y), AX_Z)
    nt = torch.where(nt > NU_FLOOR, nt, torch.full_like(nt, NU_FLOOR))
    pieces = dict(P=P, ux=ux, uy=uy, uz=uz, ub=(ubx, uby, ubz),
                  bb=(bbx, bby, bbz), D=D, cs=cs, ca=ca, nus=nus)
    return nt, pieces


def smagorinsky_rate(ux, uy, uz, D, O):
    """The Smagorinsky viscosity rate of eq. nusmag without its constant,
    [2(S_xx^2 + S_yy^2 + S_zz^2 - D^2/3 + 2(S_xy^2 + S_xz^2 + S_yz^2))]^(1/2)
    at cell centres: S_aa = ddaup(u_a); S_ab = (1/2)(ddbdn(u_a) + ddadn(u_b))
    on its edge, interpolated to the centre (up along a and b)."""
    sxx, syy, szz = O.ddxup(ux), O.ddyup(uy), O.ddzup(uz)
    sxy = O.yup(O.xup(0.5 * (O.ddydn(ux) + O.ddxdn(uy))))
    sxz = O.zup(O.xup(0.5 * (O.ddzdn(ux) + O.ddxdn(uz))))
    syz = O.zup(O.yup(0.5 * (O.ddzdn(uy) + O.ddydn(uz))))
    s2 = 2.0 * (sxx * sxx + syy * syy + szz * szz - D * D / 3.0
                + 2.0 * (sxy * sxy + sxz * sxz + syz * syz))
    return _safe_sqrt(s2)


def _safe_sqrt(s):
    """sqrt(max(s, 0)) with zero derivative where s <= 0."""
    pos = s > 0
    return torch.where(pos, torch.sqrt(torch.where(pos, s, torch.ones_like(s))), torch.zeros_like(s))


def rough_cells(rho, e, O, lim):
    """Cells where the sixth-order strain gives way to the second-order one
    (Section 3, after eq. itv): some axis's absolute second difference of
    ln rho or of ln e_m (e_m = e / rho, the energy per unit mass) exceeds
    lim (none across the ends of a wall-bounded axis)."""
    lr, le = torch.log(rho), torch.log(e / rho)
    m = None
    for a in (AX_X, AX_Y, AX_Z):
        for f in (lr, le):
            d = O.d2abs(f, a)
            m = d if m is None else torch.maximum(m, d)
    return m > lim


def strain(ux, uy, uz, O, rough=None):
    """The strain of eq. itv, (sxx, syy, szz, sxy, sxz, syz, D): diagonal and
    div u at cell centres, S_xy on the z-edge, S_xz on the y-edge, S_yz on
    the x-edge, from the sixth-order derivatives, or where `rough` (a mask
    of cells) is given, from the second-order ones wherever one of the
    cells touching the component's position is rough."""
    def d(f, ax, form, order):
        return O.stencil(f, ax, "d", form, order)
    out = []
    for order in ((6, 2) if rough is not None else (6,)):
        sxx, syy, szz = d(ux, AX_X, "up", order), d(uy, AX_Y, "up", order), d(uz, AX_Z, "up", order)
        out.append((sxx, syy, szz,
                    0.5 * (d(ux, AX_Y, "dn", order) + d(uy, AX_X, "dn", order)),
                    0.5 * (d(ux, AX_Z, "dn", order) + d(uz, AX_X, "dn", order)),
                    0.5 * (d(uy, AX_Z, "dn", order) + d(uz, AX_Y, "dn", order)),
                    sxx + syy + szz))
    if rough is None:
        return out[0]
    s6, s2 = out
    c = rough
    ze = O.any_dn(O.any_dn(c, AX_X), AX_Y)    # z-edge (i-1/2, j-1/2, k)
    ye = O.any_dn(O.any_dn(c, AX_X), AX_Z)    # y-edge (i-1/2, j, k-1/2)
    xe = O.any_dn(O.any_dn(c, AX_Y), AX_Z)    # x-edge (i, j-1/2, k-1/2)
    masks = (c, c, c, ze, ye, xe, c)
    return tuple(torch.where(mk, b, a) for mk, a, b in zip(masks, s6, s2))


def quench_factor(t, O, par):
    """The factor that multiplies a viscous stress component t (Section 6.2,
    eq. quench): q = D2 / (|t| + D2 / q_max), with D2 the sum over the three
    axes of the absolute second differences of t (zero at the end planes of
    a wall-bounded axis) and q = 0 where t and D2 both vanish; the factor is
    min(max of q over the 3x3x3 neighbourhood, q_lim).  Smooth stress
    (D2 << |t|) is reduced, a two-zone wiggle raised up to q_lim."""
    d2 = O.d2abs(t, AX_X) + O.d2abs(t, AX_Y) + O.d2abs(t, AX_Z)
    den = t.abs() + d2 / par.q_max
    pos = den > 0
    q = torch.where(pos, d2 / torch.where(pos, den, torch.ones_like(den)), torch.zeros_like(den))
    m = O.max3(O.max3(O.max3(q, AX_X), AX_Y), AX_Z)
    return torch.where(m < par.q_lim, m, torch.full_like(m, par.q_lim))


def viscosity_lengths(grid, par):
    """Length factors of eq. nuij: ((lx, ly, lz), (lxy, lxz, lyz)) with
    nu_ii = l_i <nu> and nu_ij = l_ij <nu>.  Richtmyer-Morton viscosity:
    l_i = dx_i and l_ij = max(dx_i, dx_j).  Constant viscosity (Section 6.1:
    nu_ij = const for every component): <nu> = nu_const / h_min everywhere and
    every factor is h_min, so each nu_ij is nu_const on any cell shape.
    On a stretched z axis the z spacing is the plane's own (tensors over
    the planes): its centre interval for lz, its face interval for lxz and
    lyz (the y- and x-edges sit at the faces' heights)."""
    if par.nu_const > 0:
        h = grid.hmin
        return (h, h, h), (h, h, h)
    dx, dy = grid.dx, grid.dy
    if grid.stretched:
        dzc, dzf = (d.view(-1, 1, 1) for d in grid.zintervals())
        return (dx, dy, dzc), (max(dx, dy), torch.clamp(dzf, min=dx), torch.clamp(dzf, min=dy))
    dz = grid.dz
    return (dx, dy, dz), (max(dx, dy), max(dx, dz), max(dy, dz))


def z_face_length(grid, par):
    """The z length factor of the energy-diffusion flux on the z-faces
    (eq. ediffuse): the face interval on a stretched axis."""
    if par.nu_const > 0:
        return grid.hmin
    if grid.stretched:
        return grid.zintervals()[1].view(-1, 1, 1)
    return grid.dz


def edge_viscosity(nt, grid, par, O=None):
    """Off-diagonal viscosities of eq. nuij on the cell edges (nxy on z-edges,
    nxz on y-edges, nyz on x-edges): the length factor times the exponential
    of the two-axis interpolation of ln <nu> (the paper averages ln nu for
    the off-diagonal components)."""
    O = O or grid.ops()
    _, (lxy, lxz, lyz) = viscosity_lengths(grid, par)
    lnt = torch.log(nt)
    nxy = lxy * torch.exp(O.ydn(O.xdn(lnt)))
    nxz = lxz * torch.exp(O.zdn(O.xdn(lnt)))
    nyz = lyz * torch.exp(O.zdn(O.ydn(lnt)))
    return nxy, nxz, nyz


def newton_cooling(rho, e, par):
    """Newtonian heating/cooling at cell centres (eq. NewtonCool), as a rate
    of the energy per volume: the energy per unit mass e_m = e / rho relaxes
    to e_cool on the time scale t_cool, so Q = -rho (e_m - e_cool) / t_cool.
    Optional density factor (eq. rhocool), with r = rho / rho_cool:
    r^2 / (1 + r^2) (cooling cut off at low density, cool_cut = 1) or
    1 / (1 + r^2) (cut off at high density, cool_cut = 2)."""
    em = e / rho
    q = -rho * (em - par.e_cool) / par.t_cool
    if par.cool_cut == 1:
        r2 = (rho / par.rho_cool) ** 2
        q = q * (r2 / (1.0 + r2))
    elif par.cool_cut == 2:
        r2 = (rho / par.rho_cool) ** 2
        q = q * (1.0 / (1.0 + r2))
    return q


def pressure_gradient_ln(P, O):
    """grad P on the faces through q = ln(P / P_aver) (eq. pressure), P_aver
    the mean of P over each z plane: for each axis a,
    exp(adn(ln P_aver)) exp(adn(q)) (ddadn(q) + ddadn(ln P_aver))."""
    lpa = torch.log(P.mean(dim=(1, 2), keepdim=True)).expand_as(P).contiguous()
    q = torch.log(P) - lpa
    out = []
    for dn, ddn in ((O.xdn, O.ddxdn), (O.ydn, O.ddydn), (O.zdn, O.ddzdn)):
        out.append(torch.exp(dn(lpa)) * torch.exp(dn(q)) * (ddn(q) + ddn(lpa)))
    return tuple(out)


def horizontal_ln_mean(em):
    """ln <e_m>_horiz of eq. ediffav: the logarithm of the mean of e_m over
    each z plane, broadcast over the plane."""
    return torch.log(em.mean(dim=(1, 2), keepdim=True))


def coriolis(px, py, pz, par, O):
    """Coriolis force on the momenta (eq. mom): -2 rho Omega x u, written
    -2 Omega x p, each component on its own face.  The other two momentum
    components reach that face by interpolation: up along their own axis
    (face to centre), then down along the driven axis (centre to face)."""
    ox, oy, oz = par.omega
    pz_x, py_x = O.xdn(O.zup(pz)), O.xdn(O.yup(py))      # at x-faces
    px_y, pz_y = O.ydn(O.xup(px)), O.ydn(O.zup(pz))      # at y-faces
    py_z, px_z = O.zdn(O.yup(py)), O.zdn(O.xup(px))      # at z-faces
    cx = -2.0 * (oy * pz_x - oz * py_x)
    cy = -2.0 * (oz * px_y - ox * pz_y)
    cz = -2.0 * (ox * py_z - oy * px_z)
    return cx, cy, cz


def rhs_nofill(f, grid, par, dt=None):
    """Time derivatives of the 8 variables (eqs. mass, mom, ien, indu, ohm,
    itv, vdiss, RMnu, nuij, ediffuse), evaluated on every plane of the array
    and then zeroed where Section 10 requires (ghost planes, wall faces)."""
    O = grid.ops()
    T = par.terms
    rho, px, py, pz, e, bx, by, bz = f
    mu = par.mu
    zero = torch.zeros_like(rho)

    # -- primitives (Section 4.1; eq. ien; ideal gas) ------------------------
    nt, pc = smoothed_viscosity(f, grid, par, O)
    P, ux, uy, uz, D = pc["P"], pc["ux"], pc["uy"], pc["uz"], pc["D"]
    em = e / rho                          # energy per unit mass
    (lx, ly, lz), _ = viscosity_lengths(grid, par)

    # -- viscosities and densities on edges (eq. nuij) -----------------------
    nxy, nxz, nyz = edge_viscosity(nt, grid, par, O)    # z-, y-, x-edges
    rxy = O.ydn(O.xdn(rho))
    rxz = O.zdn(O.xdn(rho))
    ryz = O.zdn(O.ydn(rho))

    # -- strain and viscous stress (eq. itv) ---------------------------------
    rough = rough_cells(rho, e, O, par.d2_lim) if T & T_ORDER2 else None
    sxx, syy, szz, sxy, sxz, syz, Dt = strain(ux, uy, uz, O, rough)
    if rough is None:
        Dt = D
    txx = rho * (lx * nt) * (sxx + par.c1 * Dt)
    tyy = rho * (ly * nt) * (syy + par.c1 * Dt)
    tzz = rho * (lz * nt) * (szz + par.c1 * Dt)
    txy = rxy * nxy * sxy
    txz = rxz * nxz * sxz
    tyz = ryz * nyz * syz
    if T & T_QUENCH:
        txx, tyy, tzz, txy, txz, tyz = (t * quench_factor(t, O, par)
                                        for t in (txx, tyy, tzz, txy, txz, tyz))

    # -- current and electric field (eq. ohm, J = curl B) ---------------------
    jx = O.ddydn(bz) - O.ddzdn(by)
    jy = O.ddzdn(bx) - O.ddxdn(bz)
    jz = O.ddxdn(by) - O.ddydn(bx)
    if par.eta_const > 0:
        etx = ety = etz = torch.full_like(rho, par.eta_const)
    else:
        etx, ety, etz = par.nuB * nyz, par.nuB * nxz, par.nuB * nxy
    ex, ey, ez = zero, zero, zero
    if T & T_INDUCT:
        ex = ex - (O.zdn(uy) * O.ydn(bz) - O.ydn(uz) * O.zdn(by))
        ey = ey - (O.xdn(uz) * O.zdn(bx) - O.zdn(ux) * O.xdn(bz))
        ez = ez - (O.ydn(ux) * O.xdn(by) - O.xdn(uy) * O.ydn(bx))
    if T & T_RESIST:
        ex = ex + etx * jx
        ey = ey + ety * jy
        ez = ez + etz * jz

    # -- mass (eq. mass) -------------------------------------------------------
    drho = zero
    if T & T_CONT:
        drho = -(O.ddxup(px) + O.ddyup(py) + O.ddzup(pz))

    # -- momentum (eq. mom) ---------------------------------------------------
    dpx, dpy, dpz = zero, zero, zero
    if T & T_ADV:
        dpx = dpx - (O.ddxdn(O.xup(px) * O.xup(ux))
                     + O.ddyup(O.ydn(px) * O.xdn(uy))
                     + O.ddzup(O.zdn(px) * O.xdn(uz)))
        dpy = dpy - (O.ddydn(O.yup(py) * O.yup(uy))
                     + O.ddzup(O.zdn(py) * O.ydn(uz))
                     + O.ddxup(O.xdn(py) * O.ydn(ux)))
        dpz = dpz - (O.ddzdn(O.zup(pz) * O.zup(uz))
                     + O.ddxup(O.xdn(pz) * O.zdn(ux))
                     + O.ddyup(O.ydn(pz) * O.zdn(uy)))
    if T & T_PRES:
        if T & T_LNP:
            gx, gy, gz = pressure_gradient_ln(P, O)
        else:
            gx, gy, gz = O.ddxdn(P), O.ddydn(P), O.ddzdn(P)
        dpx = dpx - gx
        dpy = dpy - gy
        dpz = dpz - gz
    if T & T_LORENTZ:
        dpx = dpx + (O.zup(jy * O.xdn(bz)) - O.yup(jz * O.xdn(by))) / mu
        dpy = dpy + (O.xup(jz * O.ydn(bx)) - O.zup(jx * O.ydn(bz))) / mu
        dpz = dpz + (O.yup(jx * O.zdn(by)) - O.xup(jy * O.zdn(bx))) / mu
    if T & T_VISC:
        dpx = dpx + O.ddxdn(txx) + O.ddyup(txy) + O.ddzup(txz)
        dpy = dpy + O.ddydn(tyy) + O.ddzup(tyz) + O.ddxup(txy)
        dpz = dpz + O.ddzdn(tzz) + O.ddxup(txz) + O.ddyup(tyz)
    if T & T_GRAV:
        dpz = dpz - O.zdn(rho) * par.gz
    if T & T_CORI:
        cx, cy, cz = coriolis(px, py, pz, par, O)
        dpx, dpy, dpz = dpx + cx, dpy + cy, dpz + cz

    # -- internal energy (eq. ien, eq. vdiss, eq. ediffuse) --------------------
    de = zero
    if T & T_ADV:
        de = de - (O.ddxup(O.xdn(e) * ux) + O.ddyup(O.ydn(e) * uy)
                   + O.ddzup(O.zdn(e) * uz))
    if T & T_PRES:
        de = de - P * D
    if T & T_VISC:
        qv = txx * sxx + tyy * syy + tzz * szz
        qv = qv + 2.0 * (O.yup(O.xup(txy * sxy)) + O.zup(O.xup(txz * sxz))
                         + O.zup(O.yup(tyz * syz)))
        de = de + qv
    if T & T_RESIST:
        qj = (O.zup(O.yup(etx * jx * jx)) + O.zup(O.xup(ety * jy * jy))
              + O.yup(O.xup(etz * jz * jz))) / mu
        de = de + qj
    if T & T_EDIFF:
        lne = torch.log(em)
        fx = par.nuE * O.xdn(rho) * (lx * O.xdn(nt)) * O.xdn(em) * O.ddxdn(lne)
        fy = par.nuE * O.ydn(rho) * (ly * O.ydn(nt)) * O.ydn(em) * O.ddydn(lne)
        lnez = lne
        if T & T_EDIFFAV:
            lnez = lne - horizontal_ln_mean(em)
        fz = par.nuE * O.zdn(rho) * (z_face_length(grid, par) * O.zdn(nt)) * O.zdn(em) * O.ddzdn(lnez)
        de = de + O.ddxup(fx) + O.ddyup(fy) + O.ddzup(fz)
    if T & T_COOL:
        de = de + newton_cooling(rho, e, par)

    # -- induction (eq. indu) ---------------------------------------------------
    dbx = -(O.ddyup(ez) - O.ddzup(ey))
    dby = -(O.ddzup(ex) - O.ddxup(ez))
    dbz = -(O.ddxup(ey) - O.ddyup(ex))
    if (T & T_DIVB) and dt:
        # div B diffusion: C_divb h_min^2 / dt grad(div B)
        divb = O.ddxup(bx) + O.ddyup(by) + O.ddzup(bz)
        kd = par.c_divb * grid.hmin ** 2 / dt
        dbx = dbx + kd * O.ddxdn(divb)
        dby = dby + kd * O.ddydn(divb)
        dbz = dbz + kd * O.ddzdn(divb)

    out = [drho, dpx, dpy, dpz, de, dbx, dby, dbz]
    if grid.wall:
        out = _zero_ghost_rhs(out, grid)
    return tuple(out)


def _zero_ghost_rhs(out, grid):
    """Section 10: time derivatives vanish in the ghost zones; the normal
    momentum on the two wall faces stays zero."""
    g0, g1, n = grid.ngz, grid.ngz + grid.nz, grid.nzt
    k = torch.arange(n, dtype=torch.float64).view(n, 1, 1)
    centred = ((k >= g0) & (k < g1)).to(torch.float64)
    zface = ((k >= g0) & (k <= g1)).to(torch.float64)
    pz_mask = ((k > g0) & (k < g1)).to(torch.float64)
    res = []
    for i, d in enumerate(out):
        if i == 3:
            res.append(d * pz_mask)
        elif i == 7:
            res.append(d * zface)
        else:
            res.append(d * centred)
    return res


def ghost_fill(f, grid):
    """Closed-wall ghost zones (Section 10 "Closed" and the ghost-zone
    description): ln rho and ln(e per mass) extrapolated linearly from the two
    nearest interior cells; energy per volume = density x energy per mass;
    parallel velocities symmetric and parallel field antisymmetric about the
    wall; normal mass flux antisymmetric (zero on the wall face, so no mass
    crosses it); normal field symmetric.  The lower wall is the face between
    ghost plane ngz-1 and interior plane ngz; the upper wall is the face at
    plane ngz+nz.  Interior values are never modified.  Periodic grids are
    returned unchanged."""
    if not grid.wall:
        return tuple(f)
    O = grid.ops()
    rho, px, py, pz, e, bx, by, bz = f
    g0, g1, n = grid.ngz, grid.ngz + grid.nz, grid.nzt
    lnr = torch.log(rho)
    lnm = torch.log(e / rho)

    def extrap(q, k):
        if k < g0:
            d = g0 - k
            return q[g0] + d * (q[g0] - q[g0 + 1])
        d = k - g1 + 1
        return q[g1 - 1] + d * (q[g1 - 1] - q[g1 - 2])

    ghosts = list(range(0, g0)) + list(range(g1, n))
    rho_p = [rho[k] for k in range(n)]
    e_p = [e[k] for k in range(n)]
    for k in ghosts:
        r = torch.exp(extrap(lnr, k))
        rho_p[k] = r
        e_p[k] = r * torch.exp(extrap(lnm, k))
    rho_n = torch.stack(rho_p)
    e_n = torch.stack(e_p)

    def mirror_c(k):          # centred-in-z partner plane
        return 2 * g0 - 1 - k if k < g0 else 2 * g1 - 1 - k

    rxn, ryn = O.xdn(rho_n), O.ydn(rho_n)
    px_p = [px[k] for k in range(n)]
    py_p = [py[k] for k in range(n)]
    bx_p = [bx[k] for k in range(n)]
    by_p = [by[k] for k in range(n)]
    for k in ghosts:
        m = mirror_c(k)
        px_p[k] = rxn[k] * (px[m] / rxn[m])
        py_p[k] = ryn[k] * (py[m] / ryn[m])
        bx_p[k] = -bx[m]
        by_p[k] = -by[m]
    pz_p = [pz[k] for k in range(n)]
    bz_p = [bz[k] for k in range(n)]
    pz_p[g0] = torch.zeros_like(pz[g0])
    pz_p[g1] = torch.zeros_like(pz[g1])
    for k in range(0, g0):
        pz_p[k] = -pz[2 * g0 - k]
        bz_p[k] = bz[2 * g0 - k]
    for k in range(g1 + 1, n):
        pz_p[k] = -pz[2 * g1 - k]
        bz_p[k] = bz[2 * g1 - k]
    return (rho_n, torch.stack(px_p), torch.stack(py_p), torch.stack(pz_p),
            e_n, torch.stack(bx_p), torch.stack(by_p), torch.stack(bz_p))


def rhs(f, grid, par, dt=None):
    """F(f): ghost zones filled first (wall grids), then rhs_nofill."""
    return rhs_nofill(ghost_fill(f, grid), grid, par, dt)


def rk3(f, rhs_fn, dt, nsteps=1, fill_fn=None):
    """Low-storage RK3 (eqs. dfdt, ddt, tupdate, tconst) at fixed dt on any
    tuple of arrays: for i = 1..3, dU <- alpha_i dU + F(f) (alpha_1 = 0, so
    dU starts as F), then f <- f + beta_i dt dU.  ``fill_fn`` (boundary
    conditions) is applied before the first evaluation and after every
    update."""
    fill = fill_fn or (lambda t: t)
    f = fill(tuple(f))
    for _ in range(nsteps):
        U = None
        for i in range(3):
            F = rhs_fn(f)
            U = list(F) if i == 0 else [ALPHA[i] * u + q for u, q in zip(U, F)]
            bdt = BETA[i] * dt
            f = fill(tuple(a + bdt * u for a, u in zip(f, U)))
    return f


def step(f, grid, par, dt, nsteps=1):
    """nsteps RK3 steps of the MHD system; ghost zones are refilled before
    every evaluation of F and after the last stage."""
    return rk3(f, lambda s: rhs_nofill(s, grid, par, dt), dt, nsteps,
               fill_fn=lambda s: ghost_fill(s, grid))


# ---------------------------------------------------------------------------
def courant(f, grid, par, dfdt=None):
    """Time step from eq. courantcond, evaluated on the interior cells:

    dt = min( Cdt  * dl_min / max(c_s + c_A + |u_perp|),
              Cdtd * dl_min / max(nu, eta * dl_max/dl_min),
              Cdtr / max(|drho/dt|/rho, |d e_m/dt|/e_m) )

    with nu the smoothed (speed-like) viscosity and eta its magnetic
    counterpart in the same units; the third limit only when ``dfdt`` (the
    time derivatives of f) is given.  Returns (dt, flat index of the cell that
    sets it, which limit: 0 wave, 1 diffusion, 2 rate)."""
    f = ghost_fill(tuple(f), grid)
    nt, pc = smoothed_viscosity(f, grid, par)
    rho, e = f[0], f[4]
    ubx, uby, ubz = pc["ub"]
    bbx, bby, bbz = pc["bb"]
    bb = _safe_norm3(bbx, bby, bbz)
    udotb = torch.where(bb > 0, (ubx * bbx + uby * bby + ubz * bbz) / torch.where(bb > 0, bb, torch.ones_like(bb)),
                        torch.zeros_like(bb))
    uu = ubx * ubx + uby * uby + ubz * ubz
    uperp = torch.sqrt(torch.clamp(uu - udotb * udotb, min=0.0))
    speed = pc["cs"] + pc["ca"] + uperp
    if par.eta_const > 0:
        eta_speed = torch.full_like(nt, par.eta_const / grid.hmin)
    else:
        eta_speed = par.nuB * nt
    diff = torch.maximum(nt, eta_speed * (grid.hmax / grid.hmin))
    sc, _ = interior_slices(grid)
    h = grid.hmin
    speed_i, diff_i = speed[sc], diff[sc]
    cand = []
    wmax = speed_i.max()
    cand.append((par.Cdt * h / wmax.item(), int(torch.argmax(speed_i)), 0))
    dmax = diff_i.max()
    cand.append((par.Cdtd * h / dmax.item(), int(torch.argmax(diff_i)), 1))
    if dfdt is not None:
        dr = (dfdt[0] / rho)[sc]
        dem = (dfdt[4] / e)[sc] - dr
        rate = torch.maximum(dr.abs(), dem.abs())
        rmax = rate.max().item()
        if rmax > 0:
            cand.append((par.Cdtr / rmax, int(torch.argmax(rate)), 2))
    return min(cand, key=lambda c: c[0])


def derivative_symbol(n, h):
    """K(theta_m) for the n Fourier modes m = 0..n-1 of a periodic axis of
    spacing h: the sixth-order staggered derivative (eq. deriv) multiplies
    the mode exp(i theta j), theta = 2 pi m / n, by i K with a half-cell
    shift, K = (2/h) sum_p d_p sin((2p - 1) theta / 2)."""
    th = 2.0 * math.pi * torch.arange(n, dtype=torch.float64) / n
    K = torch.zeros(n, dtype=torch.float64)
    for p, w in enumerate(DERIV6, start=1):
        K = K + w * torch.sin((2 * p - 1) * th / 2.0)
    return 2.0 * K / h


def divb_clean(f, grid):
    """div B cleaning (Section 3, eq. clean1, eq. clean2) of a periodic box:
    the potential phi with ddxup(ddxdn(phi)) + ddyup(ddydn(phi)) +
    ddzup(ddzdn(phi)) = div B, div B = ddxup(B_x) + ddyup(B_y) + ddzup(B_z)
    at the centres, solved in Fourier space, where the operator is
    multiplication by -(K_x^2 + K_y^2 + K_z^2) (zero only for the mean mode,
    whose phi is 0); then B_a - ddadn(phi) on the faces.  The cleaned B has
    zero discrete divergence; the other fields are returned unchanged."""
    if grid.wall:
        raise ValueError("div B cleaning in Fourier space needs a periodic box")
    O = grid.ops()
    rho, px, py, pz, e, bx, by, bz = f
    div = O.ddxup(bx) + O.ddyup(by) + O.ddzup(bz)
    nz, ny, nx = div.shape
    kx = derivative_symbol(nx, grid.dx) ** 2
    ky = derivative_symbol(ny, grid.dy) ** 2
    kz = derivative_symbol(nz, grid.dz) ** 2
    lap = -(kz.view(-1, 1, 1) + ky.view(1, -1, 1) + kx.view(1, 1, -1))
    dh = torch.fft.fftn(div)
    ph = torch.where(lap < 0, dh / torch.where(lap < 0, lap, torch.ones_like(lap)), torch.zeros_like(dh))
    phi = torch.fft.ifftn(ph).real
    return (rho, px, py, pz, e, bx - O.ddxdn(phi), by - O.ddydn(phi), bz - O.ddzdn(phi))


def stats(f, grid, par):
    """Conserved totals and diagnostics over the interior (float64):
    mass, momentum, kinetic / magnetic / internal energy, max and rms of
    div B (at centres, sum of ddaup B_a), max |B| component, max |u|, and the
    counts of non-finite values and of cells with rho <= 0 or e <= 0."""
    O = grid.ops()
    rho, px, py, pz, e, bx, by, bz = f
    # cell volumes (a plane's centre interval on a stretched z axis)
    dV = (grid.dx * grid.dy * grid.zintervals()[0]).view(-1, 1, 1)
    sc, _ = interior_slices(grid)
    out = {}
    out["mass"] = (rho * dV)[sc].sum().item()
    out["mom"] = [(q * dV)[sc].sum().item() for q in (px, py, pz)]
    ekin = 0.0
    for q, r in ((px, O.xdn(rho)), (py, O.ydn(rho)), (pz, O.zdn(rho))):
        ekin += (0.5 * q * q / r * dV)[sc].sum().item()
    out["ekin"] = ekin
    out["emag"] = sum((q * q * dV)[sc].sum().item() for q in (bx, by, bz)) / (2 * par.mu)
    out["eint"] = (e * dV)[sc].sum().item()
    divb = (O.ddxup(bx) + O.ddyup(by) + O.ddzup(bz))[sc]
    out["divb_max"] = divb.abs().max().item()
    out["divb_rms"] = math.sqrt((divb * divb).mean().item())
    out["bmax"] = max(q[sc].abs().max().item() for q in (bx, by, bz))
    umax = 0.0
    for q, r in ((px, O.xdn(rho)), (py, O.ydn(rho)), (pz, O.zdn(rho))):
        umax = max(umax, (q / r)[sc].abs().max().item())
    out["umax"] = umax
    nf = 0
    for q in f:
        nf += int((~torch.isfinite(q[sc])).sum())
    out["n_nonfinite"] = nf
    out["n_nonpositive"] = int(((rho[sc] <= 0) | (e[sc] <= 0)).sum())
    return out


# ---------------------------------------------------------------------------
def step_vjp(f, grid, par, dt, gbar, nsteps=1):
    """Discrete adjoint of ``step``: returns (df_end/df)^T gbar at fixed dt.
    Non-smooth choices: max3 routes to the first maximal cell; max(0,x),
    |v| and the viscosity floor have zero derivative on their flat side."""
    x = tuple(t.detach().clone().requires_grad_(True) for t in f)
    y = step(x, grid, par, dt, nsteps)
    g = torch.autograd.grad(y, x, grad_outputs=tuple(gbar), allow_unused=True)
    return tuple(torch.zeros_like(a) if b is None else b for a, b in zip(f, g))


def rhs_vjp(f, grid, par, wbar):
    """(dF/df)^T wbar for F = rhs_nofill (no ghost fill)."""
    x = tuple(t.detach().clone().requires_grad_(True) for t in f)
    y = rhs_nofill(x, grid, par)
    g = torch.autograd.grad(y, x, grad_outputs=tuple(wbar), allow_unused=True)
    return tuple(torch.zeros_like(a) if b is None else b for a, b in zip(f, g))
