"""Pins of the oracle's switch from sixth- to second-order derivatives in
the viscous stress (Section 3, after eq. itv; &pde d2lnr_lim) against
closed forms and brute force.

The second-order staggered derivative of a mode has the symbol
K2(k) = (2/h) sin(kh/2), the sixth-order one K6(k) = (2/h) sum_p d_p
sin((2p-1)kh/2); for a shear mode under constant viscosity the viscous force
on p_x is proportional to the strain's symbol, so switching every cell
scales it by exactly K2/K6.
"""
import itertools
import math

import numpy as np
import pytest
import torch

import oracle as O
from oracle.stagger import AX_X, AX_Y, AX_Z

D = torch.float64


def K6(k, h):
    return (2.0 / h) * sum(w * math.sin((2 * p - 1) * k * h / 2) for p, w in enumerate(O.DERIV6, 1))


def K2(k, h):
    return (2.0 / h) * math.sin(k * h / 2)


@pytest.mark.parametrize("axis", [AX_X, AX_Y, AX_Z])
@pytest.mark.parametrize("form", ["dn", "up"])
def test_second_order_derivative_of_a_mode(axis, form):
    n = 16
    g = O.Grid(n, n, n, Lx=1.1, Ly=0.9, Lz=1.3)
    Ops = g.ops()
    h = Ops.h[axis]
    k = 2 * math.pi * 3 / (n * h)
    i = torch.arange(n, dtype=D)
    shape = [1, 1, 1]
    shape[axis] = n
    f = torch.sin(k * i * h + 0.4).view(*shape).expand(n, n, n).contiguous()
    got = Ops.stencil(f, axis, "d", form, order=2)
    pos = (i - 0.5 if form == "dn" else i + 0.5) * h
    want = (K2(k, h) * torch.cos(k * pos + 0.4)).view(*shape).expand(n, n, n)
    assert torch.allclose(got, want, rtol=0, atol=1e-12 * K2(k, h))


def test_second_order_on_a_wall_axis_is_exact_for_a_line():
    """Every plane of a wall-bounded z axis (the end one by the copy rule)
    differentiates a linear profile exactly."""
    g = O.Grid(6, 6, 8, wall=True, ngz=5, Lz=0.8)
    Ops = g.ops()
    z = torch.arange(g.nzt, dtype=D).view(-1, 1, 1).expand(g.nzt, 6, 6) * g.dz
    for form in ("dn", "up"):
        got = Ops.stencil(2.5 * z + 1.0, AX_Z, "d", form, order=2)
        assert torch.allclose(got, torch.full_like(got, 2.5), rtol=1e-13, atol=0)


def test_second_order_on_a_wall_axis_for_a_cubic():
    """For z^3 the two-point staggered difference is 3 z^2 + dz^2 / 4 at its
    midpoint (a fourth-order stencil would give 3 z^2): every plane that has
    both samples, on the wall-bounded axis too."""
    g = O.Grid(6, 6, 10, wall=True, ngz=5, Lz=0.8)
    Ops = g.ops()
    n, h = g.nzt, g.dz
    zk = torch.arange(n, dtype=D) * h
    f = (zk ** 3).view(-1, 1, 1).expand(n, 6, 6).contiguous()
    up = Ops.stencil(f, AX_Z, "d", "up", order=2)[:, 0, 0]
    dn = Ops.stencil(f, AX_Z, "d", "dn", order=2)[:, 0, 0]
    mid_up = zk + 0.5 * h
    mid_dn = zk - 0.5 * h
    assert torch.allclose(up[:-1], 3 * mid_up[:-1] ** 2 + h * h / 4, rtol=1e-12, atol=1e-12)
    assert torch.allclose(dn[1:], 3 * mid_dn[1:] ** 2 + h * h / 4, rtol=1e-12, atol=1e-12)
    assert up[-1] == up[-2] and dn[0] == dn[1]


@pytest.mark.parametrize("wall", [False, True])
def test_rough_cells_by_brute_force(wall):
    nx, ny, nz = 5, 6, 7
    g = O.Grid(nx, ny, nz, wall=True, ngz=0) if wall else O.Grid(nx, ny, nz)
    gen = torch.Generator().manual_seed(5)
    rho = torch.exp(0.2 * torch.randn(nz, ny, nx, generator=gen, dtype=D))
    e = rho * torch.exp(0.15 * torch.randn(nz, ny, nx, generator=gen, dtype=D))
    lim = 0.35
    got = O.rough_cells(rho, e, g.ops(), lim).numpy()
    lr, le = np.log(rho.numpy()), np.log((e / rho).numpy())
    want = np.zeros((nz, ny, nx), dtype=bool)
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        m = 0.0
        for f in (lr, le):
            m = max(m, abs(f[k, j, (i + 1) % nx] - 2 * f[k, j, i] + f[k, j, (i - 1) % nx]))
            m = max(m, abs(f[k, (j + 1) % ny, i] - 2 * f[k, j, i] + f[k, (j - 1) % ny, i]))
            if not wall:
                m = max(m, abs(f[(k + 1) % nz, j, i] - 2 * f[k, j, i] + f[(k - 1) % nz, j, i]))
            elif 0 < k < nz - 1:
                m = max(m, abs(f[k + 1, j, i] - 2 * f[k, j, i] + f[k - 1, j, i]))
        want[k, j, i] = m > lim
    assert want.any() and not want.all()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("jump,expect", [(0.5, True), (0.2, False)])
def test_a_density_step_marks_the_two_cells_beside_it(jump, expect):
    """ln rho steps by `jump` between x-cells 3 and 4 (and back across the
    periodic end): |D2 ln rho| = jump exactly at cells 3 and 4 (and 0, 7),
    zero elsewhere; e_m is uniform."""
    n = 8
    g = O.Grid(n, 6, 6)
    lr = torch.zeros(6, 6, n, dtype=D)
    lr[..., 4:] = jump
    rho = torch.exp(lr)
    got = O.rough_cells(rho, 2.0 * rho, g.ops(), 0.3)
    cols = torch.zeros(n, dtype=torch.bool)
    if expect:
        cols[[0, 3, 4, 7]] = True
    assert torch.equal(got, cols.view(1, 1, n).expand(6, 6, n))


@pytest.mark.parametrize("wall", [False, True])
def test_strain_masks_follow_the_touching_cells(wall):
    """With a random mask of rough cells, each strain component takes the
    second-order value exactly where one of the cells touching its position
    (1 for a centre, 4 for an edge; those that exist on a wall axis) is
    rough, and the sixth-order value elsewhere."""
    nx, ny, nz = 6, 7, 8
    g = O.Grid(nx, ny, nz, wall=True, ngz=0) if wall else O.Grid(nx, ny, nz)
    Ops = g.ops()
    gen = torch.Generator().manual_seed(9)
    u = [torch.randn(nz, ny, nx, generator=gen, dtype=D) for _ in range(3)]
    rough = torch.rand(nz, ny, nx, generator=gen, dtype=D) < 0.15
    s6 = O.strain(*u, Ops)
    s2 = O.strain(*u, Ops, torch.ones_like(rough))
    got = O.strain(*u, Ops, rough)
    r = rough.numpy()

    def touched(k, j, i, dk, dj, di):
        for a, b, c in itertools.product(range(dk + 1), range(dj + 1), range(di + 1)):
            kk = k - a
            if wall and kk < 0:
                continue
            if r[kk % nz, (j - b) % ny, (i - c) % nx]:
                return True
        return False
    offs = [(0, 0, 0)] * 3 + [(0, 1, 1), (1, 0, 1), (1, 1, 0), (0, 0, 0)]
    for comp in range(7):
        dk, dj, di = offs[comp]
        G, A, B = got[comp].numpy(), s6[comp].numpy(), s2[comp].numpy()
        for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
            w = B if touched(k, j, i, dk, dj, di) else A
            assert G[k, j, i] == w[k, j, i], (comp, k, j, i)


def _shear(m, n=16):
    g = O.Grid(n, n, 8, Lx=1.0, Ly=1.3, Lz=0.7)
    k = 2 * math.pi * m / g.Ly
    yc = (torch.arange(n, dtype=D) + 0.5) * g.dy
    s = (g.nzt, g.ny, g.nx)
    f = [torch.full(s, 1.2, dtype=D), (1.2e-3 * torch.sin(k * yc + 0.2)).view(1, n, 1).expand(*s).contiguous()]
    f += [torch.zeros(s, dtype=D), torch.zeros(s, dtype=D), torch.full(s, 2.0, dtype=D)]
    f += [torch.zeros(s, dtype=D)] * 3
    return tuple(f), g, k


def test_rhs_switch_takes_div_u_of_the_stress_too():
    """A compression mode u_x = eps sin(k x) with c1 = -1/3: tau_xx =
    rho nu_xx (1 + c1) S_xx, so with every cell rough the viscous force on
    p_x is the sixth-order one times K2/K6 only if the stress's div u is
    second-order as well."""
    n = 16
    g = O.Grid(n, 8, 8, Lx=1.2)
    k = 2 * math.pi * 3 / g.Lx
    xf = torch.arange(n, dtype=D) * g.dx
    s = (g.nzt, g.ny, g.nx)
    f = [torch.full(s, 1.1, dtype=D), (1.1e-3 * torch.sin(k * xf)).view(1, 1, n).expand(*s).contiguous()]
    f += [torch.zeros(s, dtype=D), torch.zeros(s, dtype=D), torch.full(s, 2.0, dtype=D)]
    f += [torch.zeros(s, dtype=D)] * 3
    kw = dict(nu_const=0.02, c1=-1.0 / 3.0)
    base = O.rhs(tuple(f), g, O.Params(terms=O.T_VISC, **kw))
    all2 = O.rhs(tuple(f), g, O.Params(terms=O.T_VISC | O.T_ORDER2, d2_lim=-1.0, **kw))
    ratio = K2(k, g.dx) / K6(k, g.dx)
    assert torch.allclose(all2[1], ratio * base[1], rtol=1e-12, atol=1e-14 * float(base[1].abs().max()))


@pytest.mark.parametrize("m", [2, 5])
def test_rhs_switch_scales_a_shear_force_by_the_symbol_ratio(m):
    """Every cell rough (d2_lim < 0): the viscous force on p_x is the
    sixth-order one times K2/K6; no cell rough: bit-identical to the rhs
    without the switch."""
    f, g, k = _shear(m)
    base = O.rhs(f, g, O.Params(nu_const=0.02, terms=O.T_VISC))
    all2 = O.rhs(f, g, O.Params(nu_const=0.02, terms=O.T_VISC | O.T_ORDER2, d2_lim=-1.0))
    none = O.rhs(f, g, O.Params(nu_const=0.02, terms=O.T_VISC | O.T_ORDER2, d2_lim=1e9))
    ratio = K2(k, g.dy) / K6(k, g.dy)
    assert abs(ratio - 1.0) > 1e-3
    assert torch.allclose(all2[1], ratio * base[1], rtol=1e-12, atol=1e-14 * float(base[1].abs().max()))
    for a, b in zip(none, base):
        assert torch.equal(a, b)
