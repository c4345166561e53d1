"""Pins of the oracle's Newtonian cooling (eq. NewtonCool, eq. rhocool),
independent of its code:

* Each cell is a linear ODE for X = e - rho e_cool (rho is fixed when no
  other term acts): dX/dt = -c X with c = fac(rho) / t_cool.  One step of any
  three-stage third-order Runge-Kutta method multiplies X by the Taylor
  polynomial R(z) = 1 + z + z^2/2 + z^3/6, z = -c dt.  The printed scheme
  constants carry six digits, so R holds to about 1e-6 of z.
* The same step against the exact exp(-c dt): the error is O(z^4).
* Special densities: fac = 1/2 at rho = rho_cool for both cut-offs; 3/4 and
  1/4 at rho = sqrt(3) rho_cool.  The two cut-off factors add to 1.
* A state at e_m = e_cool is a fixed point; cooling adds to the other terms
  without changing them.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O


def _rest_state(rho_vals, em_vals, shape=(6, 6, 6)):
    rng = np.random.default_rng(3)
    n = int(np.prod(shape))
    rho = torch.tensor(rng.choice(rho_vals, n), dtype=torch.float64).reshape(shape)
    em = torch.tensor(rng.choice(em_vals, n), dtype=torch.float64).reshape(shape)
    z = torch.zeros(shape, dtype=torch.float64)
    return (rho, z.clone(), z.clone(), z.clone(), rho * em, z.clone(), z.clone(), z.clone())


def _par(cut, **kw):
    base = dict(terms=O.T_COOL, e_cool=1.7, t_cool=0.25, rho_cool=0.8, cool_cut=cut)
    base.update(kw)
    return O.Params(**base)


def _fac(rho, par):
    r2 = (rho / par.rho_cool) ** 2
    return {0: torch.ones_like(rho), 1: r2 / (1 + r2), 2: 1 / (1 + r2)}[par.cool_cut]


@pytest.mark.parametrize("cut", [0, 1, 2])
def test_one_step_is_the_rk3_polynomial(cut):
    grid = O.Grid(6, 6, 6)
    par = _par(cut)
    f = _rest_state([0.3, 0.8, 1.1, 2.5], [0.9, 1.7, 2.6, 4.0])
    dt = 0.05
    g = O.step(f, grid, par, dt, 1)
    rho = f[0]
    X0 = f[4] - rho * par.e_cool
    X1 = g[4] - rho * par.e_cool
    z = -_fac(rho, par) * dt / par.t_cool
    R = 1 + z + z * z / 2 + z ** 3 / 6
    assert torch.allclose(X1, R * X0, rtol=0, atol=2e-6 * float(X0.abs().max()))
    # against the exact decay, to third order
    ex = torch.exp(z) * X0
    assert float((X1 - ex).abs().max()) <= 0.05 * float((z.abs() ** 4 * X0.abs()).max()) + 2e-6
    # nothing else moves
    for v in (0, 1, 2, 3, 5, 6, 7):
        assert torch.equal(g[v], f[v])


def test_special_densities():
    grid = O.Grid(6, 6, 6)
    rc = 0.8
    rho_vals = [rc, math.sqrt(3) * rc]
    f = _rest_state(rho_vals, [2.7])
    q = {cut: O.rhs(f, grid, _par(cut, rho_cool=rc))[4] for cut in (0, 1, 2)}
    at1 = torch.isclose(f[0], torch.tensor(rc, dtype=torch.float64))
    at3 = ~at1
    assert at1.any() and at3.any()
    for cut in (1, 2):
        assert torch.allclose(q[cut][at1], 0.5 * q[0][at1], rtol=1e-14, atol=0)
    assert torch.allclose(q[1][at3], 0.75 * q[0][at3], rtol=1e-14, atol=0)
    assert torch.allclose(q[2][at3], 0.25 * q[0][at3], rtol=1e-14, atol=0)
    assert torch.allclose(q[1] + q[2], q[0], rtol=1e-14, atol=0)
    # the rate itself: rho (e_cool - e_m) / t_cool with e_m = 2.7
    assert torch.allclose(q[0], f[0] * (1.7 - 2.7) / 0.25, rtol=1e-14, atol=0)


def test_fixed_point():
    grid = O.Grid(6, 6, 6)
    f = _rest_state([0.4, 1.3], [1.7])
    for cut in (0, 1, 2):
        assert float(O.rhs(f, grid, _par(cut))[4].abs().max()) < 1e-15


def test_cooling_adds_to_the_other_terms():
    from paper_2405_02483_amd import inputs
    from tests.helpers import grid_params
    f, box, prm = inputs.turbulent(n=8, seed=5, kmax=2.0)
    ft = tuple(torch.from_numpy(a.copy()) for a in f)
    g, p = grid_params(box, prm, e_cool=0.6, t_cool=0.3, rho_cool=1.0, cool_cut=1)
    from dataclasses import replace
    base = O.rhs(ft, g, replace(p, terms=O.T_ALL))
    both = O.rhs(ft, g, replace(p, terms=O.T_ALL | O.T_COOL))
    cool = O.rhs(ft, g, replace(p, terms=O.T_COOL))
    for v in range(8):
        if v == 4:
            assert torch.allclose(both[4], base[4] + cool[4], rtol=1e-12, atol=1e-12)
        else:
            assert torch.equal(both[v], base[v])
