"""Pins of the oracle's pressure gradient through ln(P / P_aver)
(eq. pressure), independent of its code:

* An exponential atmosphere P = P0 exp(-z / H), uniform in the plane: ln P
  is linear in z, so the sixth-order derivative and interpolation of the
  logs are exact and the face gradient is exactly -P(z_f) / H; the plain
  sixth-order derivative of P is not (its error is of order (dz/H)^6).
* P constant on each plane: the x and y gradients vanish exactly.
* P = P_aver(z) (1 + small in-plane fluctuation): the x gradient is the
  log-derivative form P_f d ln P / dx, checked against the derivative of
  the closed-form fluctuation to sixth order.
"""
import math

import torch

import oracle as O

N = 16


def _state(P):
    shape = P.shape
    one = torch.ones(shape, dtype=torch.float64)
    zero = torch.zeros(shape, dtype=torch.float64)
    gamma = 5.0 / 3.0
    return (one, zero, zero, zero, P / (gamma - 1.0), zero, zero, zero)


def _rates(f, terms):
    out = O.rhs(f, O.Grid(N, N, N), O.Params(terms=terms))
    return -out[1], -out[2], -out[3]          # the gradient: -dp/dt with only T_PRES


def test_exponential_atmosphere_is_exact():
    H = 0.3
    i = torch.arange(N, dtype=torch.float64)
    zc = ((i + 0.5) / N).reshape(N, 1, 1).expand(N, N, N)
    P = 2.0 * torch.exp(-zc / H)
    f = _state(P)
    # periodic z: use the interior planes only, away from the wrap
    gx, gy, gz = _rates(f, O.T_PRES | O.T_LNP)
    zf = (i / N).reshape(N, 1, 1).expand(N, N, N)
    want = -2.0 * torch.exp(-zf / H) / H
    inner = slice(4, N - 3)
    assert float((gz[inner] - want[inner]).abs().max()) < 1e-11 * float(want.abs().max())
    assert float(gx.abs().max()) < 1e-14 and float(gy.abs().max()) < 1e-14
    _, _, plain = _rates(f, O.T_PRES)
    assert float((plain[inner] - want[inner]).abs().max()) > 1e-8 * float(want.abs().max())


def test_plane_constant_pressure_has_no_horizontal_gradient():
    i = torch.arange(N, dtype=torch.float64)
    zc = ((i + 0.5) / N).reshape(N, 1, 1).expand(N, N, N)
    P = 1.0 + 0.5 * torch.sin(2 * math.pi * zc)
    gx, gy, _ = _rates(_state(P), O.T_PRES | O.T_LNP)
    assert float(gx.abs().max()) < 1e-14 and float(gy.abs().max()) < 1e-14


def test_in_plane_fluctuation_log_derivative():
    i = torch.arange(N, dtype=torch.float64)
    x = ((i + 0.5) / N).reshape(1, 1, N).expand(N, N, N)
    zc = ((i + 0.5) / N).reshape(N, 1, 1).expand(N, N, N)
    a = 0.05
    P = (1.0 + 0.3 * zc) * (1.0 + a * torch.sin(2 * math.pi * x))
    gx, _, _ = _rates(_state(P), O.T_PRES | O.T_LNP)
    xf = (i / N).reshape(1, 1, N).expand(N, N, N)
    # P_f d ln P/dx at the x-face, with the sixth-order error of the stencils
    want = (1.0 + 0.3 * zc) * a * 2 * math.pi * torch.cos(2 * math.pi * xf)
    assert float((gx - want).abs().max()) < 2e-5 * float(want.abs().max())
