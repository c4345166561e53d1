"""The Coriolis force (eq. mom) in the library, through the C ABI: the
right-hand side, the RK step and the step adjoint against the float64
oracle (periodic and closed-wall boxes, every tile shape for the RHS, with
and without Newtonian cooling), a checkpointed rollout's gradient with both
terms, and the rotation of a uniform state on the GPU without the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2405_02483_amd import inputs
from tests.helpers import grid_params, interior, rel_errors, to_cpu64

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
OMEGA = (0.35, -0.6, 1.1)


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


def _over(cool=False):
    from paper_2405_02483_amd.lib import T_ALL, T_CORI, T_COOL
    o = dict(omega=OMEGA, terms=T_ALL | T_CORI)
    if cool:
        o.update(terms=T_ALL | T_CORI | T_COOL, e_cool=0.9, t_cool=0.7, rho_cool=1.1, cool_cut=2)
    return o


def _walled_errors(got, want, f, box, prm):
    g2, p2 = grid_params(box, prm, terms=O.T_GRAV)
    grav = interior(O.rhs(to_cpu64(f), g2, p2), box)
    got, want = interior(got, box), interior(want, box)
    return [float(torch.linalg.norm(a.double().cpu() - b)) /
            max(float(torch.linalg.norm(b)), float(torch.linalg.norm(c)), 1e-300)
            for a, b, c in zip(got, want, grav)]


@pytest.mark.parametrize("case", ["turb_ragged", "strat"])
@pytest.mark.parametrize("cool", [False, True])
def test_rhs_with_coriolis_all_tiles_f64(case, cool):
    from paper_2405_02483_amd.lib import TILES
    f, box, prm = _case(case)
    over = _over(cool)
    g, p = grid_params(box, prm, **over)
    want = O.rhs(to_cpu64(f), g, p)
    ctx = _ctx(box, prm, torch.float64, **over)
    fd = ctx.upload([f])
    first = None
    for tile in TILES:
        for pers in (0, 1):
            ctx.set_launch(tile, pers)
            got = ctx.box_view(ctx.rhs(fd), 0)
            errs = (_walled_errors(got, want, f, box, prm) if box.get("wall")
                    else rel_errors(got, want))
            assert max(errs) < TOL64, (tile, pers, errs)
            if first is None:
                first = [t.clone() for t in got]
            else:
                for a, b in zip(first, got):
                    assert torch.equal(a, b), (tile, pers)
    ctx.close()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, TOL64), (torch.float32, 1e-5)])
@pytest.mark.parametrize("case", ["turb_ragged", "strat"])
def test_step_with_coriolis(dtype, tol, case):
    f, box, prm = _case(case)
    over = _over()
    g, p = grid_params(box, prm, **over)
    ft = to_cpu64(f)
    dt = 0.5 * O.courant(ft, g, p)[0]
    ctx = _ctx(box, prm, dtype, **over)
    fd = ctx.upload([f])
    ctx.step(fd, dt, 2)
    want = O.step(ft, g, p, dt, 2)
    got = ctx.box_view(fd, 0)
    if box.get("wall"):
        got, want = interior(got, box), interior(want, box)
    errs = rel_errors(got, want)
    assert max(errs) < tol, errs
    ctx.close()


def test_uniform_state_rotates_f64():
    """Coriolis alone on a uniform state: one RK3 step applies the Taylor
    polynomial of the matrix of p -> -2 Omega x p (the interpolations are
    exact on a constant), to the printed digits of the scheme."""
    from paper_2405_02483_amd.lib import T_CORI
    n = 10
    p0 = np.array([0.4, -0.25, 0.7])
    one = np.ones((n, n, n))
    f = [1.3 * one, p0[0] * one, p0[1] * one, p0[2] * one, 2.0 * one, 0 * one, 0 * one, 0 * one]
    prm = dict(gamma=5 / 3, terms=T_CORI, omega=OMEGA)
    ctx = _ctx(dict(nx=n, ny=n, nz=n), prm, torch.float64)
    dt = 0.1
    fd = ctx.upload([f])
    ctx.step(fd, dt, 1)
    got = [t.double().cpu().numpy() for t in ctx.box_view(fd, 0)]
    wx, wy, wz = OMEGA
    W = np.array([[0, -wz, wy], [wz, 0, -wx], [-wy, wx, 0]])
    hA = -2.0 * dt * W
    M = np.eye(3) + hA + hA @ hA / 2 + hA @ hA @ hA / 6
    want = M @ p0
    for a in range(3):
        assert np.max(np.abs(got[1 + a] - want[a])) < 2e-6 * np.abs(p0).max()
    for v in (0, 4, 5, 6, 7):
        assert np.array_equal(got[v], np.asarray(f[v]).reshape(got[v].shape))
    ctx.close()


@pytest.mark.parametrize("cool", [False, True])
def test_step_adjoint_with_coriolis_f64(cool):
    f, box, prm = _case("turb_ragged")
    over = _over(cool)
    g, p = grid_params(box, prm, **over)
    ft = to_cpu64(f)
    dt = 0.5 * O.courant(ft, g, p)[0]
    rng = np.random.default_rng(41)
    gbar = [rng.standard_normal(a.shape) for a in f]
    ctx = _ctx(box, prm, torch.float64, **over)
    got = ctx.box_view(ctx.step_adjoint(ctx.upload([f]), dt, ctx.upload([gbar])), 0)
    want = O.step_vjp(ft, g, p, dt, to_cpu64(gbar))
    errs = rel_errors(got, want)
    assert max(errs) < 1e-10, errs
    ctx.close()


def test_rollout_with_coriolis_and_cooling_f64():
    """A 3-step checkpointed rollout with both optional terms that have an
    adjoint: its gradient against the oracle's discrete adjoint."""
    from paper_2405_02483_amd.rollout import rollout
    f, box, prm = _case("turb_ragged")
    over = _over(cool=True)
    g, p = grid_params(box, prm, **over)
    ft = to_cpu64(f)
    dt = 0.5 * O.courant(ft, g, p)[0]
    rng = np.random.default_rng(51)
    w = [rng.standard_normal(a.shape) for a in f]
    ctx = _ctx(box, prm, torch.float64, **over)
    x = [t.requires_grad_(True) for t in ctx.upload([f])]
    y = rollout(ctx, x, dt, 3, ncheck=1)
    wd = ctx.upload([w])
    grads = torch.autograd.grad(sum((a * b).sum() for a, b in zip(y, wd)), x)
    want = O.step_vjp(ft, g, p, dt, to_cpu64(w), nsteps=3)
    errs = rel_errors(ctx.box_view([t.detach() for t in grads], 0), want)
    assert max(errs) < 1e-10, errs
    ctx.close()
