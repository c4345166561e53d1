"""The library's right-hand side (float64, through the C ABI) against closed
forms, independently of the oracle: sinusoidal modes on uniform states,
compared with the operator symbols K(k) = (2/h) sum_p d_p sin((2p-1)kh/2)
(staggered derivative) and I(k) = 2 sum_p w_p cos((2p-1)kh/2) (staggered
interpolation) of eq. deriv and eq. interp.  The same modes and bounds as
the oracle's pins (tests/test_oracle_physics.py), so a dropped term, a wrong
sign, staggering or coefficient in a kernel fails here directly.
"""
import math

import pytest
import torch

import oracle as O
from paper_2405_02483_amd import inputs
from tests.test_oracle_physics import EPS, I, K, uniform_state, xs

pytestmark = pytest.mark.gpu


def _rhs(f, terms, **prm):
    """F(f) on the GPU for a periodic n^3 unit box (f: 8 CPU float64 tensors)."""
    from paper_2405_02483_amd.lib import Context
    n = f[0].shape[0]
    ctx = Context(inputs._box(n, n, n), dict(prm, terms=terms), dtype=torch.float64)
    fd = ctx.upload([[a.numpy() for a in f]])
    F = [t.view(n, n, n).cpu() for t in ctx.box_view(ctx.rhs(fd), 0)]
    ctx.close()
    return F


def _close(got, want, atol):
    return torch.allclose(got, want.expand_as(got), rtol=0, atol=atol)


def test_gravity_on_uniform_state():
    f = uniform_state(8, 1.3)
    F = _rhs(f, O.T_ALL, gz=2.5)
    assert _close(F[3], torch.full((8, 8, 8), -1.3 * 2.5, dtype=torch.float64), 1e-15 * 3.25)


def test_linear_sound_terms():
    n, m = 32, 3
    xc, xf, h = xs(n)
    k = 2 * math.pi * m
    gamma, rho0, e0 = 5.0 / 3.0, 1.2, 2.0
    P0 = (gamma - 1) * e0
    terms = O.T_CONT | O.T_ADV | O.T_PRES
    f = uniform_state(n, rho0, e=e0)
    f[1] = (rho0 * EPS * torch.sin(k * xf)).expand(n, n, n).contiguous()
    F = _rhs(f, terms, nu1=0, nu2=0, nu3=0, nuE=0)
    assert _close(F[0], -rho0 * EPS * K(k, h) * torch.cos(k * xc), 1e-12 * EPS * K(k, h))
    assert _close(F[4], -(e0 + P0) * EPS * K(k, h) * torch.cos(k * xc), 1e-6 * EPS * K(k, h))
    f = uniform_state(n, rho0, e=e0)
    f[4] = (e0 * (1 + EPS * torch.sin(k * xc))).expand(n, n, n).contiguous()
    F = _rhs(f, terms, nu1=0, nu2=0, nu3=0, nuE=0)
    assert _close(F[1], -(gamma - 1) * e0 * EPS * K(k, h) * torch.cos(k * xf), 1e-6 * EPS * e0 * K(k, h))


def test_linear_alfven_terms():
    n, m = 32, 5
    xc, xf, h = xs(n)
    k = 2 * math.pi * m
    mu, B0 = 1.7, 0.8
    terms = O.T_LORENTZ | O.T_INDUCT
    f = uniform_state(n, 1.0, b=(B0, 0.0, 0.0))
    f[6] = (EPS * torch.sin(k * xc)).expand(n, n, n).contiguous()
    F = _rhs(f, terms, mu=mu)
    assert _close(F[2], (B0 / mu) * EPS * K(k, h) * I(k, h) * torch.cos(k * xc), 1e-6 * EPS * K(k, h))
    f = uniform_state(n, 1.0, b=(B0, 0.0, 0.0))
    f[2] = (EPS * torch.sin(k * xc)).expand(n, n, n).contiguous()
    F = _rhs(f, terms, mu=mu)
    assert _close(F[6], B0 * EPS * K(k, h) * I(k, h) * torch.cos(k * xc), 1e-6 * EPS * K(k, h))


@pytest.mark.parametrize("c1", [0.0, -1.0 / 3.0])
def test_viscous_decay_rates(c1):
    n, m = 32, 4
    xc, xf, h = xs(n)
    k = 2 * math.pi * m
    nu, rho0 = 0.013, 1.4
    yc = xc.view(1, n, 1)
    f = uniform_state(n, rho0)
    f[1] = (rho0 * EPS * torch.sin(k * yc)).expand(n, n, n).contiguous()
    F = _rhs(f, O.T_VISC, nu_const=nu, c1=c1)
    want = -0.5 * nu * rho0 * EPS * K(k, h) ** 2 * torch.sin(k * yc)
    assert _close(F[1], want, 1e-9 * float(want.abs().max()))
    f = uniform_state(n, rho0)
    f[1] = (rho0 * EPS * torch.sin(k * xf)).expand(n, n, n).contiguous()
    F = _rhs(f, O.T_VISC, nu_const=nu, c1=c1)
    want = -nu * (1 + c1) * rho0 * EPS * K(k, h) ** 2 * torch.sin(k * xf)
    assert _close(F[1], want, 1e-9 * float(want.abs().max()))


def test_resistive_decay_rate():
    n, m = 32, 6
    xc, xf, h = xs(n)
    k = 2 * math.pi * m
    eta = 0.021
    f = uniform_state(n)
    f[7] = (EPS * torch.sin(k * xc)).expand(n, n, n).contiguous()
    F = _rhs(f, O.T_RESIST, eta_const=eta)
    want = -eta * EPS * K(k, h) ** 2 * torch.sin(k * xc)
    assert _close(F[7], want, 1e-9 * float(want.abs().max()))


def test_energy_diffusion_rate():
    n, m = 32, 3
    xc, xf, h = xs(n)
    k = 2 * math.pi * m
    nu, nuE, e0 = 0.011, 0.7, 1.9
    f = uniform_state(n, 1.3, e=e0)
    f[4] = (e0 * (1 + EPS * torch.sin(k * xc))).expand(n, n, n).contiguous()
    F = _rhs(f, O.T_EDIFF, nu_const=nu, nuE=nuE)
    want = -nuE * nu * e0 * EPS * K(k, h) ** 2 * torch.sin(k * xc)
    assert _close(F[4], want, 1e-6 * float(want.abs().max()))


def test_advection_is_non_dissipative():
    n, m = 32, 7
    xc, xf, h = xs(n)
    k = 2 * math.pi * m
    u0 = 0.9
    f = uniform_state(n)
    f[0] = (1.0 + EPS * torch.sin(k * xc)).expand(n, n, n).contiguous()
    f[1] = u0 * O.Grid(n, n, n).ops().xdn(f[0])
    F = _rhs(f, O.T_CONT)
    assert _close(F[0], -u0 * EPS * K(k, h) * I(k, h) * torch.cos(k * xc), 1e-12)
