"""Pins of the oracle's Coriolis force (eq. mom: -2 rho Omega x u),
independent of its code:

* A uniform state: the interpolations are exact, so dp/dt = A p with A the
  matrix of p -> -2 Omega x p, and one RK3 step is the Taylor polynomial
  I + hA + (hA)^2/2 + (hA)^3/6 applied to p (to the six printed digits of
  the scheme constants).  This fixes the signs and the factor 2.
* Momenta that vary along x only: the force on an x-face picks up the
  interpolation symbol I(k) and the half-cell shift of the down form, and
  the force on a z-face those of the up form.  This fixes which
  interpolation carries each component to which face.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O

# eq. interpcoef: the three pair weights of the sixth-order interpolation
A1, A2, A3 = 75 / 128, -25 / 256, 3 / 256


def _symbol(kh):
    return 2 * (A1 * math.cos(kh / 2) + A2 * math.cos(3 * kh / 2) + A3 * math.cos(5 * kh / 2))


def _state(n, px, py, pz):
    shape = (n, n, n)
    one = torch.ones(shape, dtype=torch.float64)
    return (1.3 * one, px, py, pz, 2.0 * one, 0 * one, 0 * one, 0 * one)


def _cross_matrix(w):
    wx, wy, wz = w
    return np.array([[0, -wz, wy], [wz, 0, -wx], [-wy, wx, 0]], dtype=np.float64)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_uniform_state_one_step_is_the_rk3_polynomial(seed):
    rng = np.random.default_rng(seed)
    om = tuple(rng.uniform(-3, 3, 3))
    p0 = rng.uniform(-1, 1, 3)
    n = 6
    one = torch.ones((n, n, n), dtype=torch.float64)
    f = _state(n, p0[0] * one, p0[1] * one, p0[2] * one)
    grid = O.Grid(n, n, n)
    par = O.Params(terms=O.T_CORI, omega=om)
    dt = 0.05
    g = O.step(f, grid, par, dt, 1)
    A = -2.0 * _cross_matrix(om)
    hA = dt * A
    M = np.eye(3) + hA + hA @ hA / 2 + hA @ hA @ hA / 6
    want = M @ p0
    for a in range(3):
        assert float((g[1 + a] - want[a]).abs().max()) < 2e-6 * np.abs(p0).max()
    for v in (0, 4, 5, 6, 7):
        assert torch.equal(g[v], f[v])


def test_momenta_varying_along_x():
    n, m = 16, 3
    h = 1.0 / n
    k = 2 * math.pi * m
    i = torch.arange(n, dtype=torch.float64)
    xc = ((i + 0.5) * h).reshape(1, 1, n).expand(n, n, n)   # centres (and y-, z-faces)
    xf = (i * h).reshape(1, 1, n).expand(n, n, n)           # x-faces
    B, C, D = 0.7, -0.4, 0.9
    px = C * torch.sin(k * xf)
    py = B * torch.sin(k * xc)
    pz = D * torch.sin(k * xc)
    om = (0.3, -1.1, 0.8)
    f = _state(n, px.clone(), py.clone(), pz.clone())
    F = O.rhs(f, O.Grid(n, n, n), O.Params(terms=O.T_CORI, omega=om))
    I = _symbol(k * h)
    ox, oy, oz = om
    # x-faces: p_y and p_z come down from the centres in x
    want_x = -2 * (oy * D - oz * B) * I * torch.sin(k * xf)
    # y-faces (x at centres): p_x comes up to the centre in x; p_z is constant in y, z
    want_y = -2 * (oz * C * I * torch.sin(k * xc) - ox * D * torch.sin(k * xc))
    # z-faces (x at centres): p_y constant along y and z; p_x comes up in x
    want_z = -2 * (ox * B * torch.sin(k * xc) - oy * C * I * torch.sin(k * xc))
    for got, want in ((F[1], want_x), (F[2], want_y), (F[3], want_z)):
        assert float((got - want).abs().max()) < 1e-13
