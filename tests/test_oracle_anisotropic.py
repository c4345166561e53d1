"""Pins of the oracle's viscosity length factors (eq. nuij), its log
averaging of the off-diagonal viscosity, the rate limit of the Courant step
(eq. courantcond) and the conserved totals, on cells with dx != dy != dz.

Each test compares with a closed form that the paper and the mathematics
fix, so that a linear instead of logarithmic edge average, a min instead of
max of two spacings, a wrong diagonal length, d ln e in place of d ln e_m in
the rate limit, or a centre density in the kinetic energy fails one of
them.  Mode tests use the operator symbol K(k, h) of eq. deriv:
ddup(dddn(sin)) = -K^2 sin, with K(k, h) = (2/h) sum_p d_p sin((2p-1)kh/2).
"""
import math

import pytest
import torch

import oracle as O

D = torch.float64
EPS = 1e-6


def K(k, h):
    return (2.0 / h) * sum(w * math.sin((2 * p - 1) * k * h / 2)
                           for p, w in enumerate(O.DERIV6, 1))


def centres(n, L):
    h = L / n
    return (torch.arange(n, dtype=D) + 0.5) * h, torch.arange(n, dtype=D) * h, h


def uniform(g, rho=1.3, p=(0.0, 0.0, 0.0), e=2.1, b=(0.0, 0.0, 0.0)):
    s = (g.nzt, g.ny, g.nx)
    return [torch.full(s, v, dtype=D) for v in (rho, *p, e, *b)]


AG = dict(nx=24, ny=20, nz=16, Lx=1.3, Ly=0.7, Lz=1.1)   # dx, dy, dz all different


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("box", [AG, dict(nx=16, ny=24, nz=20, Lx=0.6, Ly=1.2, Lz=1.5)])
def test_edge_viscosity_is_exact_for_an_exponential(box):
    """eq. nuij averages ln nu for the off-diagonal components.  With
    <nu> = exp(a x + b y + c z), ln <nu> is linear, the sixth-order
    interpolation of a linear function is exact, so each edge viscosity is
    max(dx_i, dx_j) exp(a x_e + b y_e + c z_e) at the edge position to
    rounding.  A linear average of <nu> itself is off by the interpolation
    error of an exponential (about 1e-4 here)."""
    g = O.Grid(**box)
    p = O.Params()
    xc, xf, dx = centres(g.nx, g.Lx)
    yc, yf, dy = centres(g.ny, g.Ly)
    zc, zf, dz = centres(g.nz, g.Lz)
    a, b, c = 0.45 / dx, -0.35 / dy, 0.3 / dz
    X = lambda v: v.view(1, 1, -1)
    Y = lambda v: v.view(1, -1, 1)
    Z = lambda v: v.view(-1, 1, 1)
    nt = torch.exp(a * X(xc) + b * Y(yc) + c * Z(zc)).expand(g.nz, g.ny, g.nx).contiguous()
    nxy, nxz, nyz = O.edge_viscosity(nt, g, p)
    want_xy = max(dx, dy) * torch.exp(a * X(xf) + b * Y(yf) + c * Z(zc))
    want_xz = max(dx, dz) * torch.exp(a * X(xf) + b * Y(yc) + c * Z(zf))
    want_yz = max(dy, dz) * torch.exp(a * X(xc) + b * Y(yf) + c * Z(zf))
    s = slice(3, -3)   # the stencils of the inner cells do not wrap
    for got, want in ((nxy, want_xy), (nxz, want_xz), (nyz, want_yz)):
        w = want.expand_as(got)[s, s, s]
        rel = ((got[s, s, s] - w) / w).abs().max().item()
        assert rel < 1e-13, rel
    # a linear average of <nu> is distinguishable at this resolution
    lin = max(dx, dy) * g.ops().ydn(g.ops().xdn(nt))
    w = want_xy.expand_as(lin)[s, s, s]
    assert ((lin[s, s, s] - w) / w).abs().max().item() > 1e-6


def test_viscosity_lengths():
    """eq. nuij: nu_ii = dx_i <nu>, nu_ij = max(dx_i, dx_j) <nu>; with a
    constant viscosity every factor is h_min (so nu_ij = nu_const)."""
    g = O.Grid(**AG)
    (lx, ly, lz), (lxy, lxz, lyz) = O.viscosity_lengths(g, O.Params())
    assert (lx, ly, lz) == (g.dx, g.dy, g.dz)
    assert (lxy, lxz, lyz) == (max(g.dx, g.dy), max(g.dx, g.dz), max(g.dy, g.dz))
    assert O.viscosity_lengths(g, O.Params(nu_const=0.01)) == ((g.hmin,) * 3, (g.hmin,) * 3)


# ---------------------------------------------------------------------------
def _rm_params(**over):
    """Richtmyer-Morton viscosity that is uniform on the modes below:
    nu = nu3 (c_s + c_A) with B = 0 and no |u| or shock term."""
    kw = dict(nu1=0.0, nu2=0.0, nu3=0.05, terms=O.T_VISC)
    kw.update(over)
    return O.Params(**kw)


def _nu_tilde(f, g, p):
    nt, _ = O.smoothed_viscosity(f, g, p)
    return float(nt.mean()), float((nt - nt.mean()).abs().max())


@pytest.mark.parametrize("shape", [(16, 32, 8), (32, 16, 8)])
def test_shear_decay_uses_the_larger_spacing(shape):
    """Shear u_x = eps sin(k y): dp_x/dt = ddyup(tau_xy) with
    tau_xy = rho nu_xy S_xy, so the rate is -(1/2) rho max(dx, dy) <nu> K_y^2
    (eq. itv, eq. nuij).  Both orientations of the anisotropy are run, so
    min(dx, dy) fails one of them."""
    nx, ny, nz = shape
    g = O.Grid(nx, ny, nz)
    p = _rm_params()
    rho0, m = 1.3, 3
    k = 2 * math.pi * m
    yc, _, dy = centres(ny, 1.0)
    f = uniform(g, rho0)
    f[1] = (rho0 * EPS * torch.sin(k * yc)).view(1, ny, 1).expand(nz, ny, nx).contiguous()
    nt, spread = _nu_tilde(f, g, p)
    assert spread < 1e-15
    F = O.rhs(f, g, p)
    want = -0.5 * rho0 * max(g.dx, g.dy) * nt * K(k, dy) ** 2 * EPS * torch.sin(k * yc)
    want = want.view(1, ny, 1).expand_as(F[1])
    assert torch.allclose(F[1], want, rtol=0, atol=1e-10 * float(want.abs().max()))
    assert float(F[2].abs().max()) < 1e-12 * float(want.abs().max())


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_compressive_decay_uses_the_own_spacing(axis):
    """Compression along axis a, u_a = eps sin(k x_a) on the faces:
    dp_a/dt = ddadn(tau_aa), tau_aa = rho dx_a <nu> S_aa, so the rate is
    -rho dx_a <nu> K_a^2 (eq. itv with c1 = 0, eq. nuij)."""
    g = O.Grid(**AG)
    p = _rm_params()
    rho0, m = 1.3, 2
    n, L = [(g.nx, g.Lx), (g.ny, g.Ly), (g.nz, g.Lz)][axis]
    k = 2 * math.pi * m / L
    _, xf, h = centres(n, L)
    view = [(1, 1, n), (1, n, 1), (n, 1, 1)][axis]
    f = uniform(g, rho0)
    f[1 + axis] = (rho0 * EPS * torch.sin(k * xf)).view(*view).expand(g.nz, g.ny, g.nx).contiguous()
    nt, _ = _nu_tilde(f, g, p)
    F = O.rhs(f, g, p)
    want = (-rho0 * h * nt * K(k, h) ** 2 * EPS * torch.sin(k * xf)).view(*view).expand_as(F[1 + axis])
    assert torch.allclose(F[1 + axis], want, rtol=0, atol=1e-10 * float(want.abs().max()))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_constant_viscosity_on_any_cell_shape(axis):
    """Section 6.1: a constant viscosity means nu_ij = const for every
    component, whatever the cell shape: compression along any axis decays
    at -nu K_a^2 and shear at -(nu/2) K^2."""
    g = O.Grid(**AG)
    nu, rho0, m = 0.013, 1.3, 2
    p = O.Params(nu_const=nu, terms=O.T_VISC)
    n, L = [(g.nx, g.Lx), (g.ny, g.Ly), (g.nz, g.Lz)][axis]
    k = 2 * math.pi * m / L
    xc, xf, h = centres(n, L)
    view = [(1, 1, n), (1, n, 1), (n, 1, 1)][axis]
    f = uniform(g, rho0)
    f[1 + axis] = (rho0 * EPS * torch.sin(k * xf)).view(*view).expand(g.nz, g.ny, g.nx).contiguous()
    F = O.rhs(f, g, p)
    want = (-rho0 * nu * K(k, h) ** 2 * EPS * torch.sin(k * xf)).view(*view).expand_as(F[1 + axis])
    assert torch.allclose(F[1 + axis], want, rtol=0, atol=1e-10 * float(want.abs().max()))
    # shear of the next component along this axis: u_b = eps sin(k x_a)
    b = (axis + 1) % 3
    f = uniform(g, rho0)
    f[1 + b] = (rho0 * EPS * torch.sin(k * xc)).view(*view).expand(g.nz, g.ny, g.nx).contiguous()
    F = O.rhs(f, g, p)
    want = (-0.5 * rho0 * nu * K(k, h) ** 2 * EPS * torch.sin(k * xc)).view(*view).expand_as(F[1 + b])
    assert torch.allclose(F[1 + b], want, rtol=0, atol=1e-10 * float(want.abs().max()))


@pytest.mark.parametrize("const", [False, True])
def test_energy_diffusion_uses_the_own_spacing(const):
    """eq. ediffuse with nu_yy = dy <nu> (or nu_const): uniform rho,
    e = e0 (1 + eps sin(k y)) relaxes as de/dt = -nuE nu_yy e0 eps K_y^2
    sin(k y), to first order in eps."""
    g = O.Grid(**AG)
    nuE, rho0, e0, m = 0.7, 1.3, 2.1, 2
    p = O.Params(nu_const=0.011, nuE=nuE, terms=O.T_EDIFF) if const else \
        _rm_params(nuE=nuE, terms=O.T_EDIFF)
    k = 2 * math.pi * m / g.Ly
    yc, _, dy = centres(g.ny, g.Ly)
    f = uniform(g, rho0, e=e0)
    f[4] = (e0 * (1 + EPS * torch.sin(k * yc))).view(1, g.ny, 1).expand(g.nz, g.ny, g.nx).contiguous()
    nu_yy = 0.011 if const else dy * _nu_tilde(uniform(g, rho0, e=e0), g, p)[0]
    F = O.rhs(f, g, p)
    want = (-nuE * nu_yy * e0 * EPS * K(k, dy) ** 2 * torch.sin(k * yc)).view(1, g.ny, 1).expand_as(F[4])
    assert torch.allclose(F[4], want, rtol=0, atol=1e-5 * float(want.abs().max()))


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("a,b", [(40.0, 130.0), (-40.0, 50.0)])
def test_courant_rate_limit_closed_form(a, b):
    """eq. courantcond's rate limit: Cdtr / max(|d ln rho/dt|, |d ln e_m/dt|)
    with e_m = e/rho, so d ln e_m/dt = d ln e/dt - d ln rho/dt.  A uniform
    state at rest with drho/dt = a rho and de/dt = b e gives
    Cdtr / max(|a|, |b - a|)."""
    g = O.Grid(8, 8, 8)
    p = O.Params()
    f = uniform(g)
    dfdt = [torch.zeros_like(x) for x in f]
    dfdt[0] = a * f[0]
    dfdt[4] = b * f[4]
    dt, idx, which = O.courant(f, g, p, dfdt)
    assert which == 2
    assert math.isclose(dt, p.Cdtr / max(abs(a), abs(b - a)), rel_tol=1e-14)


def test_courant_anisotropic_cells():
    """eq. courantcond on cells dx > dy > dz: the wave and diffusion limits
    take dl_min, and the magnetic diffusion speed is scaled by
    dl_max / dl_min."""
    g = O.Grid(8, 12, 16)
    p = O.Params(nu1=0.03, nu2=0.0, nu3=0.05, nuB=1.5, Cdt=0.4, Cdtd=0.6)
    rho, e, uy, bx = 1.3, 2.1, 0.4, 0.6
    f = uniform(g, rho, (0, rho * uy, 0), e, (bx, 0, 0))
    cs = math.sqrt(p.gamma * (p.gamma - 1) * e / rho)
    ca = bx / math.sqrt(rho)
    h, ratio = 1.0 / 16, 2.0
    nu = 0.03 * uy + 0.05 * (cs + ca)
    dtw = 0.4 * h / (cs + ca + uy)
    dtd = 0.6 * h / max(nu, 1.5 * nu * ratio)
    dt, idx, which = O.courant(f, g, p)
    assert math.isclose(dt, min(dtw, dtd), rel_tol=1e-14)
    assert which == (0 if dtw < dtd else 1)


# ---------------------------------------------------------------------------
def test_stats_closed_forms():
    """Totals over a periodic box with density varying along x and a
    uniform velocity u0 and field B0: p_a = adn(rho) u0_a, so the kinetic
    energy sum over faces of p_a^2 / (2 adn rho) dV is |u0|^2 M / 2, with M
    the mass (an interpolation keeps the periodic sum).  The magnetic energy
    is |B0|^2 V / (2 mu), max |u_a| and max |B_a| are the largest
    components, and div B vanishes."""
    g = O.Grid(**AG)
    p = O.Params(mu=1.7)
    Ops = g.ops()
    xc, _, dx = centres(g.nx, g.Lx)
    rho = (1.3 * (1 + 0.2 * torch.sin(2 * math.pi * xc / g.Lx))).view(1, 1, -1).expand(g.nz, g.ny, g.nx).contiguous()
    u0, b0, e0 = (0.3, -0.2, 0.5), (0.4, 0.7, -0.6), 2.1
    f = [rho, Ops.xdn(rho) * u0[0], Ops.ydn(rho) * u0[1], Ops.zdn(rho) * u0[2],
         torch.full_like(rho, e0)] + [torch.full_like(rho, v) for v in b0]
    s = O.stats(f, g, p)
    V = g.Lx * g.Ly * g.Lz
    M = float(rho.sum()) * g.dx * g.dy * g.dz
    assert math.isclose(s["mass"], M, rel_tol=1e-14)
    assert math.isclose(s["ekin"], 0.5 * sum(u * u for u in u0) * M, rel_tol=1e-13)
    assert math.isclose(s["emag"], sum(b * b for b in b0) * V / (2 * p.mu), rel_tol=1e-13)
    assert math.isclose(s["eint"], e0 * V, rel_tol=1e-13)
    for a in range(3):
        assert math.isclose(s["mom"][a], u0[a] * M, rel_tol=1e-12)
    assert math.isclose(s["umax"], 0.5, rel_tol=1e-14)
    assert s["bmax"] == 0.7
    assert s["divb_max"] < 1e-14 and s["divb_rms"] < 1e-14
    assert s["n_nonfinite"] == 0 and s["n_nonpositive"] == 0
