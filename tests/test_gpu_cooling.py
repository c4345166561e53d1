"""Newtonian cooling (eq. NewtonCool, eq. rhocool) in the library, through
the C ABI: the right-hand side, the RK step and the step adjoint against
the float64 oracle with every cut-off, and the per-cell RK3 polynomial on
the GPU without the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2405_02483_amd import inputs
from tests.helpers import grid_params, interior, rel_errors, to_cpu64

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
COOL = dict(e_cool=0.9, t_cool=0.7, rho_cool=1.1)


def _ctx(box, prm, dtype, **over):
    from paper_2405_02483_amd.lib import Context
    p = dict(prm)
    p.update(over)
    return Context(box, p, dtype=dtype)


def _case(name):
    if name == "turb_ragged":
        f, box, prm = inputs.turbulent(n=24, seed=2)
        f = [a[:, :22, :20].copy() for a in f]
        return f, dict(box, nx=20, ny=22, nz=24, Lx=20 / 24, Ly=22 / 24), prm
    return inputs.stratified(12, 10, 24, seed=3)


def _over(cut):
    from paper_2405_02483_amd.lib import T_ALL, T_COOL
    return dict(COOL, cool_cut=cut, terms=T_ALL | T_COOL)


@pytest.mark.parametrize("case", ["turb_ragged", "strat"])
@pytest.mark.parametrize("cut", [0, 1, 2])
def test_rhs_with_cooling_f64(case, cut):
    f, box, prm = _case(case)
    over = _over(cut)
    ctx = _ctx(box, prm, torch.float64, **over)
    got = ctx.box_view(ctx.rhs(ctx.upload([f])), 0)
    g, p = grid_params(box, prm, **over)
    want = O.rhs(to_cpu64(f), g, p)
    if box.get("wall"):
        # the hydrostatic z momentum rate is a small residual; judge it
        # against the gravity term (as the other walled comparisons do)
        g2, p2 = grid_params(box, prm, terms=O.T_GRAV)
        grav = interior(O.rhs(to_cpu64(f), g2, p2), box)
        got, want = interior(got, box), interior(want, box)
        errs = [float(torch.linalg.norm(a.double().cpu() - b)) /
                max(float(torch.linalg.norm(b)), float(torch.linalg.norm(c)), 1e-300)
                for a, b, c in zip(got, want, grav)]
    else:
        errs = rel_errors(got, want)
    assert max(errs) < TOL64, errs
    ctx.close()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, TOL64), (torch.float32, 1e-5)])
@pytest.mark.parametrize("cut", [0, 1, 2])
def test_step_with_cooling(dtype, tol, cut):
    f, box, prm = _case("strat")
    over = _over(cut)
    g, p = grid_params(box, prm, **over)
    ft = to_cpu64(f)
    dt = 0.5 * O.courant(ft, g, p)[0]
    ctx = _ctx(box, prm, dtype, **over)
    fd = ctx.upload([f])
    ctx.step(fd, dt, 2)
    want = O.step(ft, g, p, dt, 2)
    errs = rel_errors(interior(ctx.box_view(fd, 0), box), interior(want, box))
    assert max(errs) < tol, errs
    ctx.close()


@pytest.mark.parametrize("cut", [0, 1, 2])
def test_cooling_alone_is_the_rk3_polynomial_f64(cut):
    """Cooling alone at rest: X = e - rho e_cool obeys dX/dt = -c X per
    cell, so one RK3 step multiplies it by 1 + z + z^2/2 + z^3/6 (z = -c
    dt, c = fac(rho) / t_cool), to the six printed digits of the scheme."""
    from paper_2405_02483_amd.lib import T_COOL
    n = 12
    rng = np.random.default_rng(21)
    rho = rng.uniform(0.3, 3.0, (n, n, n))
    e = rho * rng.uniform(0.5, 2.5, (n, n, n))
    z0 = np.zeros((n, n, n))
    f = [rho, z0, z0, z0, e, z0, z0, z0]
    box = dict(nx=n, ny=n, nz=n)
    prm = dict(gamma=5 / 3, terms=T_COOL, cool_cut=cut, **COOL)
    ctx = _ctx(box, prm, torch.float64)
    dt = 0.2
    fd = ctx.upload([f])
    ctx.step(fd, dt, 1)
    got = [t.double().cpu().numpy().reshape(n, n, n) for t in ctx.box_view(fd, 0)]
    r2 = (rho / COOL["rho_cool"]) ** 2
    fac = {0: np.ones_like(rho), 1: r2 / (1 + r2), 2: 1 / (1 + r2)}[cut]
    zz = -fac * dt / COOL["t_cool"]
    X0 = e - rho * COOL["e_cool"]
    X1 = got[4] - rho * COOL["e_cool"]
    R = 1 + zz + zz ** 2 / 2 + zz ** 3 / 6
    assert np.max(np.abs(X1 - R * X0)) <= 2e-6 * np.max(np.abs(X0))
    assert np.array_equal(got[0], rho)
    for v in (1, 2, 3, 5, 6, 7):
        assert not np.any(got[v])
    ctx.close()


@pytest.mark.parametrize("cut", [0, 1, 2])
def test_step_adjoint_with_cooling_f64(cut):
    f, box, prm = _case("turb_ragged")
    over = _over(cut)
    g, p = grid_params(box, prm, **over)
    ft = to_cpu64(f)
    dt = 0.5 * O.courant(ft, g, p)[0]
    rng = np.random.default_rng(31 + cut)
    gbar = [rng.standard_normal(a.shape) for a in f]
    ctx = _ctx(box, prm, torch.float64, **over)
    got = ctx.box_view(ctx.step_adjoint(ctx.upload([f]), dt, ctx.upload([gbar])), 0)
    want = O.step_vjp(ft, g, p, dt, to_cpu64(gbar))
    errs = rel_errors(got, want)
    assert max(errs) < 1e-10, errs
    ctx.close()
