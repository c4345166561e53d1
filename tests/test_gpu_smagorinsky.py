"""The Smagorinsky viscosity (eq. nusmag, MHD_T_SMAG) and the five-cell
maximum (Section 6.1.1, MHD_T_MAX5) of the HIP library against the float64
oracle, through the C ABI: right-hand sides, steps, the Courant step of the
reductions and the adjoint, on periodic and wall-bounded boxes, isotropic
and anisotropic cells, in every tile shape and both launch modes.

Tolerances as in the other parity tests: float64 <= 1e-12 relative L2 per
field, float32 steps <= 1e-5, adjoint <= 1e-10.
"""
import math

import pytest
import torch

import oracle as O
from paper_2405_02483_amd import inputs
from tests.helpers import grid_params, interior, rel_errors, to_cpu64

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
SMAG = O.T_SMAG
MAX5 = O.T_MAX5


def _ctx(box, prm, dtype, **over):
    from paper_2405_02483_amd.lib import Context
    p = dict(prm)
    p.update(over)
    return Context(box, p, dtype=dtype)


def _case(name):
    if name == "turb_aniso":
        f, box, prm = inputs.turbulent(n=20, seed=16, kmax=3.0)
        f = [a[:18, :, :16].copy() for a in f]
        return f, dict(box, nx=16, ny=20, nz=18, Lx=1.1, Ly=0.8, Lz=1.35), prm
    if name == "turb_ragged":
        f, box, prm = inputs.turbulent(n=24, seed=12)
        f = [a[:, :22, :20].copy() for a in f]
        return f, dict(box, nx=20, ny=22, nz=24, Lx=20 / 24, Ly=22 / 24), prm
    if name == "strat":
        return inputs.stratified(12, 10, 24, seed=13)
    if name == "strat_aniso":
        f, box, prm = inputs.stratified(14, 10, 20, seed=18)
        return f, dict(box, Lx=box["Lx"] * 1.4, Ly=box["Ly"] * 0.7), prm
    if name == "min6":
        return inputs.turbulent(n=6, seed=14, kmax=2.0)
    raise KeyError(name)


CASES = ["turb_aniso", "turb_ragged", "strat", "strat_aniso", "min6"]
TERMS = {"smag": O.T_ALL | SMAG, "max5": O.T_ALL | MAX5, "both": O.T_ALL | SMAG | MAX5}


def _rhs_errs(case, terms, dtype=torch.float64, tile=None, **over):
    f, box, prm = _case(case)
    over = dict(dict(terms=terms, c_smag=0.17), **over)
    ctx = _ctx(box, prm, dtype, **over)
    if tile:
        ctx.set_launch(*tile)
    F = ctx.box_view(ctx.rhs(ctx.upload([f])), 0)
    g, p = grid_params(box, prm, **over)
    want = O.rhs(to_cpu64(f), g, p)
    ctx.close()
    return rel_errors(F, want)


@pytest.mark.parametrize("terms", sorted(TERMS))
@pytest.mark.parametrize("case", CASES)
def test_rhs_parity_f64(case, terms):
    errs = _rhs_errs(case, TERMS[terms])
    print(case, terms, ["%.2e" % e for e in errs])
    assert max(errs) < TOL64, errs


@pytest.mark.parametrize("case", ["turb_aniso", "strat_aniso"])
def test_smagorinsky_alone_f64(case):
    """The Smagorinsky term as the only viscosity (nu1 = nu2 = nu3 = 0), so
    that the strain rate alone sets every viscous flux."""
    errs = _rhs_errs(case, O.T_VISC | O.T_EDIFF | O.T_RESIST | SMAG, nu1=0.0, nu2=0.0, nu3=0.0, c_smag=0.3)
    assert max(errs) < TOL64, errs


@pytest.mark.parametrize("tile", ["64x4", "32x8", "16x16", "16x8", "64x8", "32x16"])
@pytest.mark.parametrize("persistent", [False, True])
def test_every_launch_shape_f64(tile, persistent):
    errs = _rhs_errs("strat_aniso", TERMS["both"], tile=(tile, persistent))
    assert max(errs) < TOL64, (tile, persistent, errs)


def test_launch_shapes_give_identical_bits_f32():
    from paper_2405_02483_amd.lib import TILES
    f, box, prm = _case("turb_ragged")
    ctx = _ctx(box, prm, torch.float32, terms=TERMS["both"], c_smag=0.17)
    ref = None
    for name in TILES:
        for pers in (False, True):
            ctx.set_launch(name, pers)
            fd = ctx.upload([f])
            ctx.step(fd, 2e-3, 2)
            if ref is None:
                ref = [t.clone() for t in fd]
            else:
                for a, b in zip(fd, ref):
                    assert torch.equal(a, b), (name, pers)
    ctx.close()


def test_constant_viscosity_ignores_smagorinsky():
    """With nu_const > 0 the speed-like viscosity is nu_const / h_min
    whatever MHD_T_SMAG says: identical bits with and without it."""
    f, box, prm = _case("turb_aniso")
    out = []
    for terms in (O.T_ALL, O.T_ALL | SMAG):
        ctx = _ctx(box, prm, torch.float64, terms=terms, c_smag=0.3, nu_const=0.012)
        out.append([t.clone() for t in ctx.box_view(ctx.rhs(ctx.upload([f])), 0)])
        ctx.close()
    for a, b in zip(*out):
        assert torch.equal(a, b)


@pytest.mark.parametrize("case", ["turb_aniso", "strat"])
def test_two_steps(case):
    """Two RK3 steps with the Courant step of the oracle: float64 1e-12 and
    float32 1e-5."""
    f, box, prm = _case(case)
    prm = dict(prm, terms=TERMS["both"], c_smag=0.17)
    g, p = grid_params(box, prm)
    ft = O.ghost_fill(to_cpu64(f), g)
    dt = 0.5 * O.courant(ft, g, p)[0]
    want = O.step(ft, g, p, dt, 2)
    if box.get("wall"):
        want = interior(want, box)
    for dtype, tol in ((torch.float64, TOL64), (torch.float32, 1e-5)):
        ctx = _ctx(box, prm, dtype)
        fd = ctx.upload([f])
        ctx.step(fd, dt, 2)
        got = ctx.box_view(fd, 0)
        if box.get("wall"):
            got = interior(got, box)
        errs = rel_errors(got, want)
        assert max(errs) < tol, (dtype, errs)
        ctx.close()


@pytest.mark.parametrize("case", ["turb_aniso", "strat_aniso"])
def test_reductions_courant_step(case):
    """The Courant step, its limiting cell and kind with both options: the
    diffusive limit sees the Smagorinsky viscosity and the wider maximum."""
    f, box, prm = _case(case)
    prm = dict(prm, terms=TERMS["both"], c_smag=0.4)
    g, p = grid_params(box, prm)
    ft = O.ghost_fill(to_cpu64(f), g)
    ctx = _ctx(box, prm, torch.float64)
    fd = ctx.upload([f])
    st = ctx.reductions(fd, ctx.rhs(fd))
    dt, idx, which = O.courant(ft, g, p, dfdt=O.rhs_nofill(ft, g, p))
    assert math.isclose(st["dt"], dt, rel_tol=1e-12)
    assert st["dt_limit"] == which
    nint = box["nx"] * box["ny"]
    assert st["dt_argmax"] - box.get("ngz", 0) * nint == idx
    # and the on-device step takes the same dt
    ctx.step(fd, 0.0, 1)
    assert math.isclose(ctx.last_dt(), dt, rel_tol=1e-12)
    ctx.close()


@pytest.mark.parametrize("terms", sorted(TERMS))
def test_step_adjoint_matches_oracle_f64(terms):
    import numpy as np
    f, box, prm = _case("turb_ragged")
    over = dict(terms=TERMS[terms], c_smag=0.17)
    g, p = grid_params(box, prm, **over)
    ft = to_cpu64(f)
    dt = 0.5 * O.courant(ft, g, p)[0]
    rng = np.random.default_rng(21)
    gbar = [rng.standard_normal(a.shape) for a in f]
    ctx = _ctx(box, prm, torch.float64, **over)
    out = ctx.step_adjoint(ctx.upload([f]), dt, ctx.upload([gbar]))
    errs = rel_errors(ctx.box_view(out, 0), O.step_vjp(ft, g, p, dt, to_cpu64(gbar)))
    ctx.close()
    print(terms, ["%.2e" % e for e in errs])
    assert max(errs) < 1e-10, errs
