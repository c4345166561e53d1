"""Pins of the oracle's div B diffusion (C_divb h^2 / dt grad(div B)),
independent of its code:

* B varying along x only, B_x = A sin(k x) on the x-faces: div B is the up
  derivative, its gradient the down derivative, so the B_x rate is
  -C h^2/dt K(k)^2 A sin(k x_f) with K the derivative symbol of the printed
  coefficients.  This fixes the sign, the coefficient and the pairing of the
  two derivatives.
* A discretely solenoidal B (the discrete curl of an edge vector potential)
  has div B = 0 to rounding, so the term changes nothing.
* Without a time step (a bare right-hand side) the term is absent.
"""
import math

import torch

import oracle as O

N = 16
# eq. derivcoef: the three pair weights of the sixth-order derivative
D1, D2, D3 = 75 / 64, -25 / 384, 3 / 640


def _K(k, h):
    return 2.0 / h * (D1 * math.sin(k * h / 2) + D2 * math.sin(3 * k * h / 2) + D3 * math.sin(5 * k * h / 2))


def _state(bx, by, bz):
    one = torch.ones_like(bx)
    zero = torch.zeros_like(bx)
    return (one, zero, zero, zero, 1.5 * one, bx, by, bz)


def test_x_mode_closed_form():
    h = 1.0 / N
    k = 2 * math.pi * 3
    i = torch.arange(N, dtype=torch.float64)
    xf = (i * h).reshape(1, 1, N).expand(N, N, N)
    A = 0.7
    bx = A * torch.sin(k * xf)
    zero = torch.zeros_like(bx)
    f = _state(bx, zero.clone(), zero.clone())
    c, dt = 0.08, 2e-3
    F = O.rhs(f, O.Grid(N, N, N), O.Params(terms=O.T_DIVB, c_divb=c), dt=dt)
    want = -c * h * h / dt * _K(k, h) ** 2 * A * torch.sin(k * xf)
    assert float((F[5] - want).abs().max()) < 1e-12 * float(want.abs().max())
    assert float(F[6].abs().max()) == 0.0 and float(F[7].abs().max()) == 0.0
    # a bare right-hand side has no time step: no div B diffusion
    F0 = O.rhs(f, O.Grid(N, N, N), O.Params(terms=O.T_DIVB, c_divb=c))
    assert float(F0[5].abs().max()) == 0.0


def test_solenoidal_field_is_untouched():
    g = O.Grid(N, N, N)
    Ops = g.ops()
    torch.manual_seed(3)
    ax, ay, az = (torch.randn(N, N, N, dtype=torch.float64) for _ in range(3))
    # B = curl A with A on edges: B_x = ddyup(A_z) - ddzup(A_y), ...
    bx = Ops.ddyup(az) - Ops.ddzup(ay)
    by = Ops.ddzup(ax) - Ops.ddxup(az)
    bz = Ops.ddxup(ay) - Ops.ddyup(ax)
    f = _state(bx, by, bz)
    divb = Ops.ddxup(bx) + Ops.ddyup(by) + Ops.ddzup(bz)
    assert float(divb.abs().max()) < 1e-10 * float(bx.abs().max()) * N
    on = O.rhs(f, g, O.Params(terms=O.T_DIVB, c_divb=0.1), dt=1e-3)
    assert max(float(t.abs().max()) for t in on[5:]) < 1e-8 * float(bx.abs().max()) * N * N
