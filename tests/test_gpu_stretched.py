"""A stretched z axis (Section 4.2: derivatives in index space times the
Jacobian, the inverse of the spline-fitted grid interval at each output)
in the HIP library against the float64 oracle, through the C ABI:
right-hand sides with every optional term, every tile shape and launch
mode, steps, the reductions (cell volumes, Courant step), a mixed
ensemble, and the uniform grid recovered from a linear map.

Bounds as in the other parity tests: float64 1e-12 relative L2 per field,
float32 steps 1e-5; in a walled box the z-momentum rate is judged against
the gravity term's size (the hydrostatic residual is small), as in the
random sweep.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from tests.helpers import grid_params, interior, rel_errors, to_cpu64

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _zmap(nz, ngz, L=1.0, a=0.35, b=-0.2):
    """Cell-centre heights: z = L s(u), u = (xi - ngz + 1/2) / nz, for the
    cubic s(u) = u + a u (1 - u) + b u^2 (1 - u), ghost planes included."""
    xi = np.arange(nz + 2 * ngz, dtype=np.float64)
    u = (xi - ngz + 0.5) / nz
    return L * (u + a * u * (1 - u) + b * u * u * (1 - u))


def _state(nx, ny, nz, seed, ngz=5, H=0.25, g=4.0, Lx=0.5, Ly=0.4, noise=2e-2, zmap=None):
    """An isothermal atmosphere at the stretched heights with seeded
    velocity, density and energy noise and a tilted uniform field."""
    rng = np.random.default_rng(seed)
    zc = _zmap(nz, ngz) if zmap is None else zmap
    nzt = nz + 2 * ngz
    gam = 5.0 / 3.0
    s = (nzt, ny, nx)
    rho = np.exp(-zc / H).reshape(-1, 1, 1) * np.exp(0.03 * rng.standard_normal(s))
    e = rho * g * H / (gam - 1.0) * np.exp(0.03 * rng.standard_normal(s))
    f = [rho, noise * rng.standard_normal(s) * rho, noise * rng.standard_normal(s) * rho,
         noise * rng.standard_normal(s) * rho, e,
         0.1 + 0.01 * rng.standard_normal(s), -0.05 + 0.01 * rng.standard_normal(s), np.full(s, 0.3)]
    box = dict(nx=nx, ny=ny, nz=nz, ngz=ngz, wall=True, Lx=Lx, Ly=Ly, Lz=1.0, zc=tuple(zc))
    prm = dict(gamma=gam, gz=g, nu1=0.02, nu2=1.0, nu3=0.02, nuE=1.0, nuB=1.0, c1=0.0)
    return [np.ascontiguousarray(a) for a in f], box, prm


def _ctx(box, prm, dtype, **over):
    from paper_2405_02483_amd.lib import Context
    p = dict(prm)
    p.update(over)
    return Context(box, p, dtype=dtype)


def _errs(got, want, box, prm, over):
    """Relative L2 per interior field; p_z against max(its norm, gravity's)."""
    g, p = grid_params(box, prm, **over)
    gi = interior(want, box)
    out = rel_errors(interior(got, box), gi)
    gg, pg = grid_params(box, prm, terms=O.T_GRAV)
    return out, gg, pg


OPTS = {
    "core": dict(terms=O.T_ALL),
    "everything": dict(terms=O.T_ALL | O.T_EDIFFAV | O.T_LNP | O.T_SMAG | O.T_MAX5 | O.T_QUENCH | O.T_ORDER2
                       | O.T_COOL | O.T_CORI, c_smag=0.15, e_cool=1.4, t_cool=0.5, omega=(0.2, 0.4, 0.9),
                       d2_lim=-1.0),
    "nu_const": dict(terms=O.T_ALL, nu_const=0.011),
}


def _rhs_parity(f, box, prm, over, dtype=torch.float64, launch=None):
    ctx = _ctx(box, prm, dtype, **over)
    if launch:
        ctx.set_launch(*launch)
    F = ctx.box_view(ctx.rhs(ctx.upload([f])), 0)
    g, p = grid_params(box, prm, **over)
    want = O.rhs(to_cpu64(f), g, p)
    ctx.close()
    wi = interior(want, box)
    gi = interior(F, box)
    gg, pg = grid_params(box, prm, terms=O.T_GRAV)
    grav = interior(O.rhs(to_cpu64(f), gg, pg), box)
    errs = []
    for a, w, gr in zip(gi, wi, grav):
        d = float(torch.linalg.norm(a.detach().to("cpu", torch.float64).reshape(w.shape) - w))
        scale = max(float(torch.linalg.norm(w)), float(torch.linalg.norm(gr)), 1e-300)
        errs.append(d / scale)
    return errs


@pytest.mark.parametrize("opts", sorted(OPTS))
@pytest.mark.parametrize("shape", [(12, 10, 24), (16, 9, 20)])
def test_rhs_parity_f64(shape, opts):
    f, box, prm = _state(*shape, seed=81 + shape[0])
    errs = _rhs_parity(f, box, prm, OPTS[opts])
    print(shape, opts, ["%.2e" % e for e in errs])
    assert max(errs) < TOL64, errs


@pytest.mark.parametrize("tile", ["64x4", "32x8", "16x16", "16x8", "64x8", "32x16"])
@pytest.mark.parametrize("persistent", [False, True])
def test_every_launch_shape_f64(tile, persistent):
    f, box, prm = _state(14, 10, 20, seed=85)
    errs = _rhs_parity(f, box, prm, OPTS["everything"], launch=(tile, persistent))
    assert max(errs) < TOL64, (tile, persistent, errs)


def test_linear_map_matches_the_uniform_box():
    """Heights on a line give the uniform grid's right-hand side (the
    spline's intervals equal dz up to rounding)."""
    nx, ny, nz, ngz = 10, 8, 16, 5
    dz = 1.0 / nz
    zlin = (np.arange(nz + 2 * ngz) - ngz + 0.5) * dz
    f, box, prm = _state(nx, ny, nz, seed=86, zmap=zlin)
    ubox = {k: v for k, v in box.items() if k != "zc"}
    a = _ctx(box, prm, torch.float64)
    b = _ctx(ubox, prm, torch.float64)
    Fa = a.box_view(a.rhs(a.upload([f])), 0)
    Fb = b.box_view(b.rhs(b.upload([f])), 0)
    for x, y in zip(interior(Fa, box), interior(Fb, box)):
        assert float((x - y).abs().max()) <= 1e-12 * float(y.abs().max() + 1e-300)
    a.close()
    b.close()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, TOL64), (torch.float32, 1e-5)])
def test_two_steps(dtype, tol):
    f, box, prm = _state(12, 10, 24, seed=87, noise=1e-2)
    g, p = grid_params(box, prm)
    ft = O.ghost_fill(to_cpu64(f), g)
    dt = 0.5 * O.courant(ft, g, p)[0]
    want = interior(O.step(ft, g, p, dt, 2), box)
    ctx = _ctx(box, prm, dtype)
    fd = ctx.upload([f])
    ctx.step(fd, dt, 2)
    got = interior(ctx.box_view(fd, 0), box)
    errs = rel_errors(got, want)
    print(dtype, ["%.2e" % e for e in errs])
    assert max(errs) < tol, errs
    ctx.close()


def test_reductions_and_courant_step():
    """Totals with the cell volumes dx dy dz_c, and the Courant step with the
    box's smallest spacing, against the oracle; the on-device step takes
    the same dt."""
    f, box, prm = _state(12, 10, 24, seed=88)
    g, p = grid_params(box, prm)
    ft = O.ghost_fill(to_cpu64(f), g)
    ctx = _ctx(box, prm, torch.float64)
    fd = ctx.upload([f])
    st = ctx.reductions(fd, ctx.rhs(fd))
    want = O.stats(ft, g, p)
    for key in ("mass", "ekin", "emag", "eint"):
        assert math.isclose(st[key], want[key], rel_tol=1e-12), (key, st[key], want[key])
    for a_ in range(3):
        assert abs(st["mom"][a_] - want["mom"][a_]) < 1e-12 * max(1.0, abs(want["mom"][a_]))
    dt, idx, which = O.courant(ft, g, p, dfdt=O.rhs_nofill(ft, g, p))
    assert math.isclose(st["dt"], dt, rel_tol=1e-12)
    assert st["dt_limit"] == which
    ctx.step(fd, 0.0, 1)
    assert math.isclose(ctx.last_dt(), O.courant(ft, g, p)[0], rel_tol=1e-12)
    ctx.close()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, TOL64), (torch.float32, 1e-5)])
def test_mixed_ensemble_step(dtype, tol):
    """A stretched walled box, a uniform walled box and a periodic box in
    one context (pass F's stretched launch serves all three): one step each
    against the oracle."""
    from paper_2405_02483_amd import inputs
    s1 = _state(10, 8, 16, seed=89, noise=1e-2)
    f2, b2, p2 = inputs.stratified(8, 10, 12, seed=90)
    f3, b3, p3 = inputs.turbulent(n=8, seed=91, kmax=2.0)
    cases = [s1, (f2, b2, p2), (f3, b3, p3)]
    prm = dict(s1[2])
    ctx = _ctx([c[1] for c in cases], prm, dtype)
    fd = ctx.upload([c[0] for c in cases])
    dt = 1e-3
    ctx.step(fd, dt, 1)
    for bi, (f, box, _) in enumerate(cases):
        g, p = grid_params(box, prm)
        want = O.step(O.ghost_fill(to_cpu64(f), g), g, p, dt, 1)
        got = ctx.box_view(fd, bi)
        if box.get("wall"):
            got, want = interior(got, box), interior(want, box)
        errs = rel_errors(got, want)
        assert max(errs) < tol, (bi, errs)
    ctx.close()
