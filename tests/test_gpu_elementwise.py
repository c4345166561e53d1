"""Element-by-element parity of the library's right-hand side and RK step
with the float64 oracle, through the C ABI.

The L2 measures of the other parity tests floor a field's norm at 1e-3 of
the largest field's, and an error confined to one plane or one tile seam
can hide in a norm.  Here every element of every field is checked, ghost
and wall planes included, against the size of what is summed there: the
sum over the term groups of |F_group| at that element (each group's
right-hand side from the oracle alone), so that small fields (the
horizontal field rates of a walled box, the hydrostatic residual of p_z) are
judged on their own scale.

Bound per element: |got - want| <= tol * S + floor, S the local sum of the
groups' magnitudes and floor = tol * 1e-3 * max(S) over the field (for
elements where every group nearly vanishes).  float64: tol = 1e-12, about
5000 units of rounding, room for sixth-order stencils of fluxes larger than
their differences (measured: at most 2e-13).  float32 right-hand side at the
float32-rounded state: tol = 5e-4 (measured 9e-5): the float32 arithmetic
rounds every flux to 6e-8, amplified by 1/(k dx) through each derivative and
by the cancellation inside a group (e.g. -grad P against the momentum flux
divergence).  RK step increments (f_end - f_start, float64): tol = 5e-11
with S = dt times the local group sum (measured 5e-12: the increment is a
difference of two states of order one).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2405_02483_amd import inputs
from tests.helpers import grid_params, interior, to_cpu64

pytestmark = pytest.mark.gpu

CORE = (O.T_CONT, O.T_ADV, O.T_PRES, O.T_VISC, O.T_LORENTZ, O.T_INDUCT, O.T_RESIST, O.T_EDIFF, O.T_GRAV)
MODS = O.T_EDIFFAV | O.T_LNP | O.T_SMAG | O.T_MAX5 | O.T_QUENCH | O.T_ORDER2
EVERYTHING = dict(terms=O.T_ALL | O.T_EDIFFAV | O.T_LNP | O.T_SMAG | O.T_MAX5 | O.T_QUENCH | O.T_ORDER2
                  | O.T_COOL | O.T_CORI, c_smag=0.15, e_cool=1.4, t_cool=0.5, omega=(0.2, 0.4, 0.9),
                  d2_lim=-1.0)


def _ctx(box, prm, dtype, **over):
    from paper_2405_02483_amd.lib import Context
    p = dict(prm)
    p.update(over)
    return Context(box, p, dtype=dtype)


def _walled(nx, ny, nz, seed, ngz=5, aniso=1.0):
    """A closed-wall atmosphere with density, energy, velocity and field
    noise (every ghost-fill rule and wall stencil active)."""
    rng = np.random.default_rng(seed)
    nzt = nz + 2 * ngz
    H, g, gam = 0.25, 4.0, 5.0 / 3.0
    zc = (np.arange(nzt) - ngz + 0.5) / nz
    s = (nzt, ny, nx)
    rho = np.exp(-zc / H).reshape(-1, 1, 1) * np.exp(0.05 * rng.standard_normal(s))
    e = rho * g * H / (gam - 1.0) * np.exp(0.05 * rng.standard_normal(s))
    f = [rho, 0.05 * rng.standard_normal(s) * rho, 0.05 * rng.standard_normal(s) * rho,
         0.05 * rng.standard_normal(s) * rho, e, 0.1 + 0.02 * rng.standard_normal(s),
         -0.05 + 0.02 * rng.standard_normal(s), 0.3 + 0.02 * rng.standard_normal(s)]
    box = dict(nx=nx, ny=ny, nz=nz, ngz=ngz, wall=True, Lx=aniso * nx / nz, Ly=ny / nz, Lz=1.0)
    prm = dict(gamma=gam, gz=g, nu1=0.02, nu2=1.0, nu3=0.02, nuE=1.0, nuB=1.0, c1=0.0)
    return [np.ascontiguousarray(a) for a in f], box, prm


def _case(name):
    if name == "ragged":
        f, box, prm = inputs.turbulent(n=24, seed=2)
        f = [a[:, :22, :20].copy() for a in f]
        return f, dict(box, nx=20, ny=22, nz=24, Lx=20 / 24, Ly=22 / 24), prm
    if name == "seams":     # several tiles in x and y, ragged in all three
        f, box, prm = inputs.turbulent(n=40, seed=3, kmax=4.0)
        f = [a[:17, :26, :40].copy() for a in f]
        return f, dict(box, nx=40, ny=26, nz=17, Lx=1.0, Ly=26 / 40, Lz=17 / 40), prm
    if name == "walled":
        return _walled(12, 10, 24, 81)
    if name == "walled_aniso":
        return _walled(14, 9, 16, 82, aniso=1.3)
    if name == "strat":     # the benchmark's atmosphere, small
        return inputs.stratified(12, 10, 24, seed=3)
    raise KeyError(name)


def _group_scale(f, box, prm, over, dt=None):
    """Sum over the term groups of |F_group| per element (oracle)."""
    terms = over.get("terms", O.T_ALL)
    mods = terms & MODS
    groups = [b | mods for b in CORE if terms & b]
    groups += [b for b in (O.T_COOL, O.T_CORI) if terms & b]
    if dt is not None and terms & O.T_DIVB:
        groups.append(O.T_DIVB)
    ft = to_cpu64(f)
    S = None
    for t in groups:
        g, p = grid_params(box, prm, **dict(over, terms=t))
        Fg = O.rhs(ft, g, p, dt) if dt is not None else O.rhs(ft, g, p)
        a = [x.abs() for x in Fg]
        S = a if S is None else [s + x for s, x in zip(S, a)]
    return S


def _element_ratio(got, want, S, tol):
    """Per field: max over elements of |got - want| / (tol S + floor)."""
    out = []
    for gv, w, s in zip(got, want, S):
        d = (gv.detach().to("cpu", torch.float64).reshape(w.shape) - w).abs()
        floor = tol * 1e-3 * float(s.max()) + 1e-300
        out.append(float((d / (tol * s + floor)).max()))
    return out


CASES = ["ragged", "seams", "walled", "walled_aniso", "strat"]


@pytest.mark.parametrize("terms", ["core", "everything"])
@pytest.mark.parametrize("case", CASES)
def test_rhs_every_element_f64(case, terms):
    f, box, prm = _case(case)
    over = dict(terms=O.T_ALL) if terms == "core" else EVERYTHING
    g, p = grid_params(box, prm, **over)
    want = O.rhs(to_cpu64(f), g, p)
    S = _group_scale(f, box, prm, over)
    ctx = _ctx(box, prm, torch.float64, **over)
    got = ctx.box_view(ctx.rhs(ctx.upload([f])), 0)
    ctx.close()
    r = _element_ratio(got, want, S, 1e-12)
    print(case, terms, ["%.2e" % x for x in r])
    assert max(r) <= 1.0, r


@pytest.mark.parametrize("case", CASES)
def test_rhs_every_element_f32(case):
    f, box, prm = _case(case)
    g, p = grid_params(box, prm)
    # the oracle at the float32-rounded state: the stored inputs' rounding
    # is the library's input, not its error
    f32 = [np.asarray(a, dtype=np.float32).astype(np.float64) for a in f]
    want = O.rhs(to_cpu64(f32), g, p)
    S = _group_scale(f32, box, prm, {})
    ctx = _ctx(box, prm, torch.float32)
    got = ctx.box_view(ctx.rhs(ctx.upload([f])), 0)
    ctx.close()
    r = _element_ratio(got, want, S, 5e-4)
    print(case, ["%.2e" % x for x in r])
    assert max(r) <= 1.0, r


@pytest.mark.parametrize("case", ["ragged", "walled", "walled_aniso"])
def test_step_increment_every_element_f64(case):
    """One RK step with every optional term (and div B diffusion, which
    needs the step's dt): f_end - f_start per element of the interior (the
    ghost planes are refilled from it)."""
    f, box, prm = _case(case)
    over = dict(EVERYTHING, terms=EVERYTHING["terms"] | O.T_DIVB, c_divb=0.08)
    g, p = grid_params(box, prm, **over)
    ft = O.ghost_fill(to_cpu64(f), g)
    dt = 0.5 * O.courant(ft, g, p)[0]
    want = [b - a for a, b in zip(ft, O.step(ft, g, p, dt))]
    S = [dt * s for s in _group_scale([a.numpy() for a in ft], box, prm, over, dt=dt)]
    ctx = _ctx(box, prm, torch.float64, **over)
    fd = ctx.upload([[a.numpy() for a in ft]])
    f0 = [t.clone() for t in ctx.box_view(fd, 0)]
    ctx.step(fd, dt, 1)
    got = [b - a for a, b in zip(f0, ctx.box_view(fd, 0))]
    ctx.close()
    if box.get("wall"):
        got, want, S = interior(got, box), interior(want, box), interior(S, box)
    r = _element_ratio(got, want, S, 5e-11)
    print(case, ["%.2e" % x for x in r])
    assert max(r) <= 1.0, r
