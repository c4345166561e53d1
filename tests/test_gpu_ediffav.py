"""Energy diffusion about the horizontal mean (eq. ediffav) in the library,
through the C ABI: the right-hand side and the RK step against the float64
oracle, in closed-wall and periodic boxes and in an ensemble (per-box plane
tables) and a plane-constant state that must not diffuse.  The adjoint
with this term is tested with the other adjoint tests."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2405_02483_amd import inputs
from tests.helpers import grid_params, interior, rel_errors, to_cpu64

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _ctx(boxes, prm, dtype, **over):
    from paper_2405_02483_amd.lib import Context
    p = dict(prm)
    p.update(over)
    return Context(boxes, p, dtype=dtype)


def _over():
    from paper_2405_02483_amd.lib import T_ALL, T_EDIFFAV
    return dict(terms=T_ALL | T_EDIFFAV)


def _ragged():
    f, box, prm = inputs.turbulent(n=24, seed=2)
    f = [a[:, :22, :20].copy() for a in f]
    return f, dict(box, nx=20, ny=22, nz=24, Lx=20 / 24, Ly=22 / 24), prm


def _strat(nx, ny, nz, seed):
    """The stratified box with an energy profile that is not isothermal and
    not uniform in the plane, so both the mean and the fluctuation form of
    the diffusion act."""
    f, box, prm = inputs.stratified(nx, ny, nz, seed=seed)
    nzt = f[4].shape[0]
    zc = (np.arange(nzt) + 0.5) / nzt
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    prof = (1.0 + 0.3 * zc)[:, None, None]
    fl = 1.0 + 0.1 * np.sin(2 * math.pi * x)[None, None, :] * np.cos(2 * math.pi * y)[None, :, None]
    f[4] = f[4] * prof * fl
    return f, box, prm


def _errors(got, want, f, box, prm):
    if not box.get("wall"):
        return rel_errors(got, want)
    g2, p2 = grid_params(box, prm, terms=O.T_GRAV)
    grav = interior(O.rhs(to_cpu64(f), g2, p2), box)
    got, want = interior(got, box), interior(want, box)
    return [float(torch.linalg.norm(a.double().cpu() - b)) /
            max(float(torch.linalg.norm(b)), float(torch.linalg.norm(c)), 1e-300)
            for a, b, c in zip(got, want, grav)]


@pytest.mark.parametrize("case", ["strat", "ragged"])
def test_rhs_ediffav_f64(case):
    f, box, prm = _strat(12, 10, 24, 3) if case == "strat" else _ragged()
    over = _over()
    g, p = grid_params(box, prm, **over)
    want = O.rhs(to_cpu64(f), g, p)
    ctx = _ctx(box, prm, torch.float64, **over)
    got = ctx.box_view(ctx.rhs(ctx.upload([f])), 0)
    errs = _errors(got, want, f, box, prm)
    assert max(errs) < TOL64, errs
    # it changes the energy rate (else this test would not test it)
    g0, p0 = grid_params(box, prm)
    plain = O.rhs(to_cpu64(f), g0, p0)[4]
    assert float((plain - want[4]).abs().max()) > 1e-6 * float(plain.abs().max())
    ctx.close()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, TOL64), (torch.float32, 1e-5)])
def test_step_ediffav_walls(dtype, tol):
    f, box, prm = _strat(12, 10, 24, 3)
    over = _over()
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


def test_ensemble_plane_tables_f64():
    """Three walled boxes of different heights in one persistent launch:
    each box's planes have their own entries in the plane-mean table."""
    cases = [_strat(nx, ny, nz, 20 + b)
             for b, (nx, ny, nz) in enumerate(((12, 10, 24), (8, 14, 13), (10, 9, 30)))]
    prm = cases[0][2]
    over = _over()
    ctx = _ctx([c[1] for c in cases], prm, torch.float64, **over)
    ctx.set_launch("32x8", 1)
    F = ctx.rhs(ctx.upload([c[0] for c in cases]))
    for b, (f, box, _) in enumerate(cases):
        g, p = grid_params(box, prm, **over)
        want = O.rhs(to_cpu64(f), g, p)
        errs = _errors(ctx.box_view(F, b), want, f, box, prm)
        assert max(errs) < TOL64, (b, errs)
    ctx.close()


def test_plane_constant_energy_does_not_diffuse_f64():
    """Energy diffusion alone, e_m constant on each plane: no flux at all
    about the plane mean (while plain diffusion moves energy along z)."""
    from paper_2405_02483_amd.lib import T_EDIFF, T_EDIFFAV
    n = 12
    z = (np.arange(n) + 0.5) / n
    em = np.broadcast_to((1.5 + 0.4 * np.sin(2 * math.pi * z))[:, None, None], (n, n, n))
    rho = np.broadcast_to((1.0 + 0.2 * np.cos(2 * math.pi * z))[:, None, None], (n, n, n))
    zero = np.zeros((n, n, n))
    f = [rho.copy(), zero, zero, zero, (rho * em).copy(), zero, zero, zero]
    box = dict(nx=n, ny=n, nz=n)
    prm = dict(gamma=5 / 3)
    rates = {}
    for name, terms in (("av", T_EDIFF | T_EDIFFAV), ("plain", T_EDIFF)):
        ctx = _ctx(box, prm, torch.float64, terms=terms)
        rates[name] = ctx.box_view(ctx.rhs(ctx.upload([f])), 0)[4].double().cpu()
        ctx.close()
    assert float(rates["plain"].abs().max()) > 1e-3
    assert float(rates["av"].abs().max()) < 1e-12 * float(rates["plain"].abs().max())
