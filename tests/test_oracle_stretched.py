"""Pins of the oracle's stretched z axis (Section 4.2: derivatives in index
space times the Jacobian, the inverse of the spline-fitted grid interval at
the derivative's centre) against closed forms and convergence.

The not-a-knot cubic spline reproduces a cubic exactly, so for a cubic map
z(xi) the grid intervals are its exact derivative, at the centres, the
faces and the extrapolated first face.  A linear map is a uniform grid.
Sixth-order index-space derivatives of f(z(xi)) converge as n^-6 when the
map is refined (z = L s(xi / n) for a fixed cubic s).  A hydrostatic
atmosphere's pressure gradient balances gravity to the same order, which
fails if the Jacobian is left out or put on the wrong stagger.  The cell
volumes dx dy dz_c make the mass an exact invariant of a step with walls.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from oracle.stagger import AX_Z

D = torch.float64


def cubic_map(n, L=1.0, a=0.35, b=-0.2):
    """z(xi) = L s(u), u = (xi + 1/2) / n, s(u) = u + a u (1 - u) + b u^2 (1 - u):
    increasing for these a, b."""
    def s(u):
        return u + a * u * (1 - u) + b * u * u * (1 - u)

    def ds(u):
        return 1 + a * (1 - 2 * u) + b * (2 * u - 3 * u * u)
    xi = np.arange(n, dtype=np.float64)
    u = (xi + 0.5) / n
    return L * s(u), (lambda x: L * ds((x + 0.5) / n) / n)


def test_spline_intervals_exact_for_a_cubic_map():
    n = 23
    zc, dz = cubic_map(n, L=2.0)
    dzc, dzf = O.zgrid_intervals(tuple(zc))
    xi = np.arange(n, dtype=np.float64)
    assert np.allclose(dzc.numpy(), dz(xi), rtol=1e-13, atol=0)
    assert np.allclose(dzf.numpy(), dz(xi - 0.5), rtol=1e-13, atol=0)


@pytest.mark.parametrize("form", ["dn", "up"])
def test_derivative_of_the_height_is_one_on_every_plane(form):
    """A quadratic map: every stencil (sixth, fourth and second order near
    the ends) differentiates the heights exactly in index space, so with
    the right Jacobian on every plane (the ends included) dz/dz = 1."""
    n = 16
    zc, dz = cubic_map(n, L=1.3, b=0.0)
    g = O.Grid(4, 4, n, wall=True, ngz=0, zc=tuple(zc))
    xi = np.arange(n, dtype=np.float64)
    zin = zc if form == "dn" else _zat(xi - 0.5, n, L=1.3, b=0.0)
    f = torch.from_numpy(zin).view(-1, 1, 1).expand(n, 4, 4).contiguous()
    got = g.ops().stencil(f, AX_Z, "d", form)[:, 0, 0]
    assert torch.allclose(got, torch.ones_like(got), rtol=0, atol=1e-13)


def test_linear_map_is_the_uniform_grid():
    from paper_2405_02483_amd import inputs
    f, box, prm = inputs.stratified(8, 6, 12, seed=7)
    g0 = O.Grid(**box)
    h = g0.dz
    zc = tuple(h * (k - g0.ngz + 0.5) for k in range(g0.nzt))
    g1 = O.Grid(**dict(box, zc=zc))
    p = O.Params(**{k: v for k, v in prm.items() if k in O.Params.__dataclass_fields__})
    ft = tuple(torch.from_numpy(a) for a in f)
    a = O.rhs(ft, g0, p)
    b = O.rhs(ft, g1, p)
    for x, y in zip(a, b):
        assert float((x - y).abs().max()) <= 1e-11 * float(x.abs().max() + 1e-30)


@pytest.mark.parametrize("form", ["up", "dn"])
def test_index_space_derivative_converges_at_sixth_order(form):
    """ddz of sin(k z) on a cubic stretched map, interior planes at least 3
    from the ends: error ratio above 40 per doubling (64 at sixth order)."""
    errs = []
    for n in (24, 48, 96):
        zc, dz = cubic_map(n, L=1.0)
        g = O.Grid(4, 4, n, wall=True, ngz=0, zc=tuple(zc))
        Ops = g.ops()
        z = torch.from_numpy(zc)
        kk = 2.0 * math.pi * 1.5
        xi = np.arange(n, dtype=np.float64)
        if form == "up":      # input on faces (xi - 1/2), output at centres
            zin = torch.from_numpy(_zat(xi - 0.5, n))
            zout = z
        else:                 # input at centres, output on faces
            zin = z
            zout = torch.from_numpy(_zat(xi - 0.5, n))
        f = torch.sin(kk * zin).view(-1, 1, 1).expand(n, 4, 4).contiguous()
        got = Ops.stencil(f, AX_Z, "d", form)[:, 0, 0]
        want = kk * torch.cos(kk * zout)
        errs.append(float((got - want)[4:-4].abs().max()))
    assert errs[0] / errs[1] > 40 and errs[1] / errs[2] > 40, errs


def _zat(x, n, L=1.0, a=0.35, b=-0.2):
    u = (x + 0.5) / n
    return L * (u + a * u * (1 - u) + b * u * u * (1 - u))


def _hydrostatic(n, H=0.25, g=4.0, ngz=5):
    """Isothermal atmosphere at rest on a stretched z of n interior planes
    (heights from the cubic map, continued smoothly into the ghost planes),
    P = rho g H, e = P / (gamma - 1)."""
    nzt = n + 2 * ngz
    xi = np.arange(nzt, dtype=np.float64) - ngz
    zc = _zat(xi, n)
    gam = 5.0 / 3.0
    rho = np.exp(-zc / H)
    e = rho * g * H / (gam - 1.0)
    s = (nzt, 6, 6)
    f = [np.broadcast_to(rho.reshape(-1, 1, 1), s).copy(), np.zeros(s), np.zeros(s), np.zeros(s),
         np.broadcast_to(e.reshape(-1, 1, 1), s).copy(), np.zeros(s), np.zeros(s), np.zeros(s)]
    grid = O.Grid(6, 6, n, ngz=ngz, wall=True, Lx=0.1, Ly=0.1, Lz=1.0, zc=tuple(zc))
    par = O.Params(gamma=gam, gz=g, terms=O.T_PRES | O.T_GRAV)
    return tuple(torch.from_numpy(a) for a in f), grid, par


def test_hydrostatic_balance_converges():
    res = []
    for n in (64, 128):      # 4 scale heights: 32 planes are still pre-asymptotic
        f, g, p = _hydrostatic(n)
        F = O.rhs_nofill(f, g, p)
        sc = slice(g.ngz + 4, g.ngz + g.nz - 4)
        res.append(float(F[3][sc].abs().max()) / (float(f[0].max()) * p.gz))
    assert res[0] < 1e-8 and res[0] / res[1] > 30, res
    # leaving the Jacobian out breaks the balance at order one
    f, g, p = _hydrostatic(32)
    g_wrong = O.Grid(6, 6, 32, ngz=5, wall=True, Lx=0.1, Ly=0.1, Lz=1.0)
    F = O.rhs_nofill(f, g_wrong, p)
    sc = slice(10, 32)
    assert float(F[3][sc].abs().max()) / (float(f[0].max()) * p.gz) > 1e-2


def test_mass_is_invariant_with_cell_volumes():
    from paper_2405_02483_amd import inputs
    f, box, prm = inputs.stratified(8, 8, 16, seed=9, noise=0.05)
    nzt = 16 + 2 * box["ngz"]
    zc, _ = cubic_map(nzt, L=1.0 * nzt / 16)
    g = O.Grid(**dict(box, zc=tuple(zc - zc[box["ngz"]] + 0.5 * (zc[1] - zc[0]))))
    p = O.Params(**{k: v for k, v in prm.items() if k in O.Params.__dataclass_fields__})
    ft = O.ghost_fill(tuple(torch.from_numpy(a) for a in f), g)
    m0 = O.stats(ft, g, p)["mass"]
    dt = 0.5 * O.courant(ft, g, p)[0]
    f1 = O.step(ft, g, p, dt, 1)
    m1 = O.stats(O.ghost_fill(f1, g), g, p)["mass"]
    assert abs(m1 - m0) < 1e-13 * m0
    # the same sum with uniform volumes is not conserved
    dzc = g.zintervals()[0]
    sc = slice(g.ngz, g.ngz + g.nz)
    u0 = float(ft[0][sc].sum())
    u1 = float(O.ghost_fill(f1, g)[0][sc].sum())
    assert abs(u1 - u0) > 1e3 * abs(m1 - m0) / float(dzc.mean()) / (g.dx * g.dy)


def test_local_spacings_sit_at_each_quantity_s_height():
    """On a stretched z: nu_zz's length is the centre interval, the y- and
    x-edge lengths max(dx, face interval), max(dy, face interval), the
    energy-diffusion z flux's the face interval, and the shock viscosity's
    h the smallest spacing of the cell (intervals from the cubic map's
    closed-form derivative)."""
    n = 20
    zc, dz = cubic_map(n, L=2.5)
    # dx and dy inside the range of the z intervals (0.106 .. 0.169), so
    # the smallest spacing changes from plane to plane
    g = O.Grid(6, 7, n, wall=True, ngz=0, Lx=0.78, Ly=1.05, zc=tuple(zc))
    p = O.Params()
    xi = np.arange(n, dtype=np.float64)
    (lx, ly, lz), (lxy, lxz, lyz) = O.viscosity_lengths(g, p)
    assert np.allclose(lz.view(-1).numpy(), dz(xi), rtol=1e-13)
    assert np.allclose(lxz.view(-1).numpy(), np.maximum(g.dx, dz(xi - 0.5)), rtol=1e-13)
    assert np.allclose(lyz.view(-1).numpy(), np.maximum(g.dy, dz(xi - 0.5)), rtol=1e-13)
    assert np.allclose(O.z_face_length(g, p).view(-1).numpy(), dz(xi - 0.5), rtol=1e-13)
    assert lxy == max(g.dx, g.dy)
    # the shock viscosity alone: nus = h_cell max(0, -div u)
    gen = torch.Generator().manual_seed(3)
    s = (n, 7, 6)
    f = (torch.ones(s, dtype=D) * 1.2, 0.1 * torch.randn(s, generator=gen, dtype=D),
         0.1 * torch.randn(s, generator=gen, dtype=D), 0.1 * torch.randn(s, generator=gen, dtype=D),
         torch.ones(s, dtype=D) * 2.0, torch.zeros(s, dtype=D), torch.zeros(s, dtype=D), torch.zeros(s, dtype=D))
    _, pc = O.smoothed_viscosity(f, g, O.Params(nu1=0.0, nu3=0.0, nu2=1.0))
    hcell = torch.from_numpy(np.minimum(np.minimum(g.dx, g.dy), dz(xi))).view(-1, 1, 1)
    assert torch.allclose(pc["nus"], hcell * torch.clamp(-pc["D"], min=0.0), rtol=1e-13, atol=0)
