"""Quenching of the viscous stress (Section 6.2, eq. quench; MHD_T_QUENCH)
in the HIP library against the float64 oracle, through the C ABI:
right-hand sides, steps and the adjoint, on periodic and wall-bounded boxes
and anisotropic cells, in every tile shape and both launch modes, alone and
with the Smagorinsky viscosity and the five-cell maximum.

Tolerances as in the other parity tests: float64 <= 1e-12 relative L2 per
field, float32 steps <= 1e-5, adjoint <= 1e-10.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2405_02483_amd import inputs
from tests.helpers import grid_params, interior, rel_errors, to_cpu64

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
Q = O.T_QUENCH


def _ctx(box, prm, dtype, **over):
    from paper_2405_02483_amd.lib import Context
    p = dict(prm)
    p.update(over)
    return Context(box, p, dtype=dtype)


def _case(name):
    if name == "turb_aniso":
        f, box, prm = inputs.turbulent(n=20, seed=26, kmax=3.0)
        f = [a[:18, :, :16].copy() for a in f]
        return f, dict(box, nx=16, ny=20, nz=18, Lx=1.1, Ly=0.8, Lz=1.35), prm
    if name == "turb_ragged":
        f, box, prm = inputs.turbulent(n=24, seed=22)
        f = [a[:, :22, :20].copy() for a in f]
        return f, dict(box, nx=20, ny=22, nz=24, Lx=20 / 24, Ly=22 / 24), prm
    if name == "strat":
        return inputs.stratified(12, 10, 24, seed=23)
    if name == "strat_aniso":
        f, box, prm = inputs.stratified(14, 10, 20, seed=28)
        return f, dict(box, Lx=box["Lx"] * 1.4, Ly=box["Ly"] * 0.7), prm
    if name == "min6":
        return inputs.turbulent(n=6, seed=24, kmax=2.0)
    raise KeyError(name)


CASES = ["turb_aniso", "turb_ragged", "strat", "strat_aniso", "min6"]
VARIANTS = {
    "default": dict(terms=O.T_ALL | Q),
    "uncapped": dict(terms=O.T_ALL | Q, q_max=3.0, q_lim=10.0),
    "with_smag_max5": dict(terms=O.T_ALL | Q | O.T_SMAG | O.T_MAX5, c_smag=0.17, q_lim=1.5),
}


def _rhs_errs(case, over, dtype=torch.float64, launch=None):
    f, box, prm = _case(case)
    ctx = _ctx(box, prm, dtype, **over)
    if launch:
        ctx.set_launch(*launch)
    F = ctx.box_view(ctx.rhs(ctx.upload([f])), 0)
    g, p = grid_params(box, prm, **over)
    want = O.rhs(to_cpu64(f), g, p)
    ctx.close()
    return rel_errors(F, want)


@pytest.mark.parametrize("variant", sorted(VARIANTS))
@pytest.mark.parametrize("case", CASES)
def test_rhs_parity_f64(case, variant):
    errs = _rhs_errs(case, VARIANTS[variant])
    print(case, variant, ["%.2e" % e for e in errs])
    assert max(errs) < TOL64, errs


def test_quenching_changes_the_rhs():
    """The option is not a no-op on these states: the viscous force and
    heating differ from the unquenched ones by far more than rounding."""
    f, box, prm = _case("turb_aniso")
    out = []
    for terms in (O.T_VISC, O.T_VISC | Q):
        ctx = _ctx(box, prm, torch.float64, terms=terms)
        out.append([t.to("cpu", torch.float64) for t in ctx.box_view(ctx.rhs(ctx.upload([f])), 0)])
        ctx.close()
    errs = rel_errors(out[1], out[0])
    assert max(errs[1:5]) > 1e-2, errs


def test_without_viscosity_quenching_is_a_no_op():
    f, box, prm = _case("strat")
    out = []
    for terms in (O.T_ALL & ~O.T_VISC, (O.T_ALL & ~O.T_VISC) | Q):
        ctx = _ctx(box, prm, torch.float64, terms=terms)
        out.append([t.clone() for t in ctx.box_view(ctx.rhs(ctx.upload([f])), 0)])
        ctx.close()
    for a, b in zip(*out):
        assert torch.equal(a, b)


@pytest.mark.parametrize("tile", ["64x4", "32x8", "16x16", "16x8", "64x8", "32x16"])
@pytest.mark.parametrize("persistent", [False, True])
def test_every_launch_shape_f64(tile, persistent):
    errs = _rhs_errs("strat_aniso", VARIANTS["with_smag_max5"], launch=(tile, persistent))
    assert max(errs) < TOL64, (tile, persistent, errs)


def test_launch_shapes_give_identical_bits_f32():
    from paper_2405_02483_amd.lib import TILES
    f, box, prm = _case("turb_ragged")
    ctx = _ctx(box, prm, torch.float32, **VARIANTS["default"])
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


@pytest.mark.parametrize("case", ["turb_aniso", "strat"])
def test_two_steps(case):
    f, box, prm = _case(case)
    prm = dict(prm, **VARIANTS["default"])
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


@pytest.mark.parametrize("variant", ["default", "uncapped", "with_smag_max5"])
def test_step_adjoint_matches_oracle_f64(variant):
    f, box, prm = _case("turb_ragged")
    over = VARIANTS[variant]
    g, p = grid_params(box, prm, **over)
    ft = to_cpu64(f)
    dt = 0.5 * O.courant(ft, g, p)[0]
    rng = np.random.default_rng(31)
    gbar = [rng.standard_normal(a.shape) for a in f]
    ctx = _ctx(box, prm, torch.float64, **over)
    out = ctx.step_adjoint(ctx.upload([f]), dt, ctx.upload([gbar]))
    errs = rel_errors(ctx.box_view(out, 0), O.step_vjp(ft, g, p, dt, to_cpu64(gbar)))
    ctx.close()
    print(variant, ["%.2e" % e for e in errs])
    assert max(errs) < 1e-10, errs
