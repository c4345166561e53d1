"""Pressure gradient through ln(P / P_aver) (eq. pressure) in the library,
through the C ABI: the right-hand side and the RK step against the float64
oracle (closed-wall and periodic boxes, an ensemble with per-box plane
tables) and the exact gradient of an exponential atmosphere on the GPU
alone.  The adjoint with this term is tested with the other adjoint tests."""
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
    from paper_2405_02483_amd.lib import T_ALL, T_LNP
    return dict(terms=T_ALL | T_LNP)


def _strat(nx, ny, nz, seed):
    """The stratified box with pressure fluctuations in the plane."""
    f, box, prm = inputs.stratified(nx, ny, nz, seed=seed)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    fl = 1.0 + 0.05 * np.sin(2 * math.pi * x)[None, None, :] * np.cos(2 * math.pi * y)[None, :, None]
    f[4] = f[4] * fl
    return f, box, prm


def _ragged():
    f, box, prm = inputs.turbulent(n=24, seed=2)
    f = [a[:, :22, :20].copy() for a in f]
    return f, dict(box, nx=20, ny=22, nz=24, Lx=20 / 24, Ly=22 / 24), prm


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
def test_rhs_lnp_f64(case):
    f, box, prm = _strat(12, 10, 24, 3) if case == "strat" else _ragged()
    over = _over()
    g, p = grid_params(box, prm, **over)
    want = O.rhs(to_cpu64(f), g, p)
    ctx = _ctx(box, prm, torch.float64, **over)
    got = ctx.box_view(ctx.rhs(ctx.upload([f])), 0)
    errs = _errors(got, want, f, box, prm)
    assert max(errs) < TOL64, errs
    ctx.close()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, TOL64), (torch.float32, 1e-5)])
def test_step_lnp_walls(dtype, tol):
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
    cases = [_strat(nx, ny, nz, 40 + b) for b, (nx, ny, nz) in enumerate(((12, 10, 24), (8, 14, 13)))]
    cases.append(_ragged())
    prm = cases[0][2]
    over = _over()
    ctx = _ctx([c[1] for c in cases], prm, torch.float64, **over)
    ctx.set_launch("16x16", 1)
    F = ctx.rhs(ctx.upload([c[0] for c in cases]))
    for b, (f, box, _) in enumerate(cases):
        g, p = grid_params(box, prm, **over)
        want = O.rhs(to_cpu64(f), g, p)
        errs = _errors(ctx.box_view(F, b), want, f, box, prm)
        assert max(errs) < TOL64, (b, errs)
    ctx.close()


def test_exponential_atmosphere_gradient_is_exact_f64():
    """The static isothermal atmosphere (P = rho = exp(-z / H), extrapolated
    into the ghost planes in ln rho): with the pressure term alone, the
    p_z rate on every interior face is P(z_f) / H to rounding, which the
    plain sixth-order derivative misses by its truncation error."""
    from paper_2405_02483_amd.lib import T_PRES, T_LNP
    f, box, prm = inputs.stratified(8, 8, 32, seed=3, noise=0.0)
    H = 1.0 / 4.0
    ngz, nz = box["ngz"], box["nz"]
    zf = (np.arange(nz + 2 * ngz) - ngz) / nz
    want = np.exp(-zf / H) / H
    inner = slice(ngz + 1, ngz + nz)
    rates = {}
    for name, terms in (("lnp", T_PRES | T_LNP), ("plain", T_PRES)):
        ctx = _ctx(box, prm, torch.float64, terms=terms)
        rates[name] = ctx.box_view(ctx.rhs(ctx.upload([f])), 0)[3].double().cpu().numpy()
        ctx.close()
    w = np.broadcast_to(want[:, None, None], rates["lnp"].shape)
    err = np.max(np.abs(rates["lnp"][inner] - w[inner])) / np.max(np.abs(w[inner]))
    plain = np.max(np.abs(rates["plain"][inner] - w[inner])) / np.max(np.abs(w[inner]))
    assert err < 1e-13, err
    assert plain > 100 * max(err, 1e-16), (plain, err)
