"""div B diffusion (c_divb h^2 / dt grad(div B)) in the library, through the
C ABI: RK steps against the float64 oracle (periodic and closed-wall boxes,
a mixed persistent ensemble), its absence from a bare right-hand side and
the per-step decay of an x mode on the GPU alone.  The adjoint with this term
is tested with the other adjoint tests."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2405_02483_amd import inputs
from tests.helpers import grid_params, interior, rel_errors, to_cpu64

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
CDIVB = 0.08


def _ctx(boxes, prm, dtype, **over):
    from paper_2405_02483_amd.lib import Context
    p = dict(prm)
    p.update(over)
    return Context(boxes, p, dtype=dtype)


def _over():
    from paper_2405_02483_amd.lib import T_ALL, T_DIVB
    return dict(terms=T_ALL | T_DIVB, c_divb=CDIVB)


def _ragged():
    f, box, prm = inputs.turbulent(n=24, seed=2)
    f = [a[:, :22, :20].copy() for a in f]
    return f, dict(box, nx=20, ny=22, nz=24, Lx=20 / 24, Ly=22 / 24), prm


def _strat(nx, ny, nz, seed):
    """The stratified box with a non-solenoidal perturbation of B_x."""
    f, box, prm = inputs.stratified(nx, ny, nz, seed=seed)
    rng = np.random.default_rng(seed)
    f[5] = f[5] + 0.02 * rng.standard_normal(f[5].shape)
    return f, box, prm


def _step(f, box, prm, dtype, nsteps=2):
    over = _over()
    g, p = grid_params(box, prm, **over)
    ft = to_cpu64(f)
    dt = 0.5 * O.courant(ft, g, p)[0]
    ctx = _ctx(box, prm, dtype, **over)
    fd = ctx.upload([f])
    ctx.step(fd, dt, nsteps)
    want = O.step(ft, g, p, dt, nsteps)
    got = ctx.box_view(fd, 0)
    ctx.close()
    if box.get("wall"):
        return interior(got, box), interior(want, box)
    return got, want


@pytest.mark.parametrize("case", ["ragged", "strat"])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, TOL64), (torch.float32, 1e-5)])
def test_step_divb(case, dtype, tol):
    f, box, prm = _ragged() if case == "ragged" else _strat(12, 10, 24, 3)
    got, want = _step(f, box, prm, dtype)
    errs = rel_errors(got, want)
    assert max(errs) < tol, errs
    # the term acts (else this would not test it)
    g0, p0 = grid_params(box, prm)
    ft = to_cpu64(f)
    dt = 0.5 * O.courant(ft, *grid_params(box, prm, **_over()))[0]
    plain = O.step(ft, g0, p0, dt, 2)
    if box.get("wall"):
        plain = interior(plain, box)
    assert float((plain[5] - want[5]).abs().max()) > 1e-9


def test_mixed_ensemble_persistent_f64():
    cases = [_ragged(), _strat(8, 14, 13, 7), _strat(12, 10, 24, 3)]
    prm = cases[1][2]
    over = _over()
    dt = 0.5 * min(O.courant(to_cpu64(c[0]), *grid_params(c[1], prm, **over))[0] for c in cases)
    ctx = _ctx([c[1] for c in cases], prm, torch.float64, **over)
    ctx.set_launch("32x8", 1)
    fd = ctx.upload([c[0] for c in cases])
    ctx.step(fd, dt, 1)
    for b, (f, box, _) in enumerate(cases):
        g, p = grid_params(box, prm, **over)
        want = O.step(to_cpu64(f), g, p, dt, 1)
        got = ctx.box_view(fd, b)
        if box.get("wall"):
            got, want = interior(got, box), interior(want, box)
        errs = rel_errors(got, want)
        assert max(errs) < TOL64, (b, errs)
    ctx.close()


def test_bare_rhs_leaves_it_out():
    from paper_2405_02483_amd.lib import T_ALL
    f, box, prm = _ragged()
    out = {}
    for name, over in (("on", _over()), ("off", dict(terms=T_ALL))):
        ctx = _ctx(box, prm, torch.float64, **over)
        out[name] = [t.clone() for t in ctx.box_view(ctx.rhs(ctx.upload([f])), 0)]
        ctx.close()
    for a, b in zip(out["on"], out["off"]):
        assert torch.equal(a, b)


def test_x_mode_decays_by_the_rk3_polynomial_f64():
    """div B diffusion alone on B_x = A sin(k x): each step multiplies it by
    R(z) = 1 + z + z^2/2 + z^3/6 with z = -c_divb h^2 K(k)^2 (the dt of
    the coefficient cancels the step's), K the derivative symbol."""
    from paper_2405_02483_amd.lib import T_DIVB
    n = 16
    h = 1.0 / n
    k = 2 * math.pi * 3
    xf = np.arange(n) * h
    A = 0.7
    one = np.ones((n, n, n))
    zero = np.zeros((n, n, n))
    bx = A * np.broadcast_to(np.sin(k * xf)[None, None, :], (n, n, n)).copy()
    f = [one, zero, zero, zero, 1.5 * one, bx, zero, zero]
    ctx = _ctx(dict(nx=n, ny=n, nz=n), dict(gamma=5 / 3), torch.float64, terms=T_DIVB, c_divb=CDIVB)
    fd = ctx.upload([f])
    ctx.step(fd, 1e-3, 1)
    got = ctx.box_view(fd, 0)[5].double().cpu().numpy().reshape(n, n, n)
    ctx.close()
    d1, d2, d3 = 75 / 64, -25 / 384, 3 / 640
    K = 2 / h * (d1 * math.sin(k * h / 2) + d2 * math.sin(3 * k * h / 2) + d3 * math.sin(5 * k * h / 2))
    z = -CDIVB * h * h * K * K
    R = 1 + z + z * z / 2 + z ** 3 / 6
    assert np.max(np.abs(got - R * bx)) < 2e-6 * A


def test_step_with_device_courant_dt_f64():
    """dt = 0: the library takes the Courant dt on the device, and the div B
    coefficient uses that dt (read back with last_dt for the oracle)."""
    f, box, prm = _strat(12, 10, 24, 3)
    over = _over()
    ctx = _ctx(box, prm, torch.float64, **over)
    fd = ctx.upload([f])
    ctx.step(fd, 0.0, 1)
    dt = ctx.last_dt()
    g, p = grid_params(box, prm, **over)
    want = O.step(to_cpu64(f), g, p, dt, 1)
    errs = rel_errors(interior(ctx.box_view(fd, 0), box), interior(want, box))
    assert max(errs) < TOL64, errs
    ctx.close()
