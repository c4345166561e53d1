"""Pins of the oracle's quenching of the viscous stress (Section 6.2,
eq. quench) against closed forms and brute force.

For a single mode t = A sin(k x + phi) the second difference is exactly
-(2 - 2 cos kh) t, so q = c / (1 + c / q_max) with c = 2 - 2 cos kh at every
cell, and the factor is min(q, q_lim): about (kh)^2 for a smooth mode, and
for the two-zone wiggle (kh = pi, c = 4) q = 4 / (1 + 4 / q_max), capped at
q_lim.
"""
import itertools
import math

import numpy as np
import pytest
import torch

import oracle as O
from oracle.stagger import AX_X, AX_Y, AX_Z

D = torch.float64


def factor(kh, qmax=8.0, qlim=2.0):
    c = 2.0 - 2.0 * math.cos(kh)
    return min(c / (1.0 + c / qmax), qlim)


@pytest.mark.parametrize("axis", [AX_X, AX_Y, AX_Z])
@pytest.mark.parametrize("m", [1, 3, 6])
def test_single_mode_closed_form(axis, m):
    n = 12
    g = O.Grid(n, n, n)
    Ops = g.ops()
    par = O.Params()
    k = 2 * math.pi * m / n                       # per cell: kh
    i = torch.arange(n, dtype=D)
    shape = [1, 1, 1]
    shape[axis] = n
    t = (0.7 * torch.sin(k * i + 0.3)).view(*shape).expand(n, n, n).contiguous()
    got = O.quench_factor(t, Ops, par)
    assert torch.allclose(got, torch.full_like(got, factor(k)), rtol=1e-13, atol=0)
    if m == 6:   # the two-zone wiggle: q = 8/3 capped at q_lim = 2
        assert factor(k) == 2.0


def test_smooth_mode_is_reduced_like_kh_squared():
    n = 64
    g = O.Grid(n, 4, 4)
    k = 2 * math.pi / n
    t = torch.sin(k * torch.arange(n, dtype=D) + 0.1).view(1, 1, n).expand(4, 4, n).contiguous()
    f = O.quench_factor(t, g.ops(), O.Params())
    assert abs(float(f.mean()) / k ** 2 - 1.0) < 0.01


@pytest.mark.parametrize("qmax,qlim", [(8.0, 2.0), (3.0, 10.0)])
def test_wiggle_factor_and_parameters(qmax, qlim):
    """A wiggle along y: q = 4 / (1 + 4 / q_max), capped at q_lim."""
    n = 8
    g = O.Grid(n, n, n)
    t = ((-1.0) ** torch.arange(n, dtype=D)).view(1, n, 1).expand(n, n, n).contiguous() * 2.5
    f = O.quench_factor(t, g.ops(), O.Params(q_max=qmax, q_lim=qlim))
    want = min(4.0 / (1.0 + 4.0 / qmax), qlim)
    assert torch.allclose(f, torch.full_like(f, want), rtol=1e-14, atol=0)


@pytest.mark.parametrize("qmax,qlim", [(5.0, 10.0), (8.0, 2.0)])
@pytest.mark.parametrize("wall", [False, True])
def test_brute_force_on_a_small_random_field(wall, qmax, qlim):
    """Loops over the cells: the sum of absolute second differences (none
    across the ends of a wall-bounded z axis), q, the maximum over the
    available 3x3x3 neighbours, and the cap (q_lim above q_max: never
    reached, so every q counts)."""
    nx, ny, nz = 5, 6, 7
    g = O.Grid(nx, ny, nz, wall=wall, ngz=0) if wall else O.Grid(nx, ny, nz)
    gen = torch.Generator().manual_seed(3)
    t = torch.randn(nz, ny, nx, generator=gen, dtype=D)
    t[2, 3, 1] = 0.0
    par = O.Params(q_max=qmax, q_lim=qlim)
    got = O.quench_factor(t, g.ops(), par).numpy()
    a = t.numpy()
    q = np.zeros_like(a)
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        d2 = abs(a[k, j, (i + 1) % nx] - 2 * a[k, j, i] + a[k, j, (i - 1) % nx])
        d2 += abs(a[k, (j + 1) % ny, i] - 2 * a[k, j, i] + a[k, (j - 1) % ny, i])
        if not wall:
            d2 += abs(a[(k + 1) % nz, j, i] - 2 * a[k, j, i] + a[(k - 1) % nz, j, i])
        elif 0 < k < nz - 1:
            d2 += abs(a[k + 1, j, i] - 2 * a[k, j, i] + a[k - 1, j, i])
        den = abs(a[k, j, i]) + d2 / par.q_max
        q[k, j, i] = d2 / den if den > 0 else 0.0
    want = np.zeros_like(a)
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        ks = [k - 1, k, k + 1]
        ks = [x for x in ks if 0 <= x < nz] if wall else [x % nz for x in ks]
        m = max(q[kk, (j + dj) % ny, (i + di) % nx] for kk in ks for dj in (-1, 0, 1) for di in (-1, 0, 1))
        want[k, j, i] = min(m, par.q_lim)
    assert np.allclose(got, want, rtol=1e-14, atol=0)


def test_zero_stress_gives_zero_factor():
    g = O.Grid(6, 6, 6)
    f = O.quench_factor(torch.zeros(6, 6, 6, dtype=D), g.ops(), O.Params())
    assert torch.equal(f, torch.zeros_like(f))


def _shear(m, n=16):
    g = O.Grid(n, n, 8, Lx=1.0, Ly=1.3, Lz=0.7)
    k = 2 * math.pi * m / g.Ly
    yc = (torch.arange(n, dtype=D) + 0.5) * g.dy
    s = (g.nzt, g.ny, g.nx)
    rho = torch.full(s, 1.2, dtype=D)
    f = [rho, (1.2e-3 * torch.sin(k * yc + 0.2)).view(1, n, 1).expand(*s).contiguous()]
    f += [torch.zeros(s, dtype=D), torch.zeros(s, dtype=D), torch.full(s, 2.0, dtype=D)]
    f += [torch.zeros(s, dtype=D)] * 3
    return tuple(f), g, k * g.dy


@pytest.mark.parametrize("m", [2, 8])
def test_rhs_scales_stress_and_heating_by_the_factor(m):
    """A shear mode under constant viscosity: the only stress, tau_xy, is a
    single y mode, so with quenching the viscous force on p_x and the
    viscous heating are the unquenched ones times the closed-form factor
    (m = 8 is the two-zone wiggle on 16 cells)."""
    f, g, kh = _shear(m)
    p = O.Params(nu_const=0.02, terms=O.T_VISC)
    pq = O.Params(nu_const=0.02, terms=O.T_VISC | O.T_QUENCH)
    a = O.rhs(f, g, p)
    b = O.rhs(f, g, pq)
    fac = factor(kh)
    assert torch.allclose(b[1], fac * a[1], rtol=1e-12, atol=1e-14 * float(a[1].abs().max()))
    assert torch.allclose(b[4], fac * a[4], rtol=1e-12, atol=1e-14 * float(a[4].abs().max()))
    assert float(a[1].abs().max()) > 0 and float(a[4].abs().max()) > 0


def test_uniform_state_is_unchanged():
    g = O.Grid(6, 6, 6)
    s = (6, 6, 6)
    f = tuple(torch.full(s, v, dtype=D) for v in (1.0, 0.1, -0.2, 0.3, 1.5, 0.2, 0.1, -0.1))
    a = O.rhs(f, g, O.Params())
    b = O.rhs(f, g, O.Params(terms=O.T_ALL | O.T_QUENCH))
    for x, y in zip(a, b):
        assert torch.isfinite(y).all()
        assert torch.equal(x, y)
