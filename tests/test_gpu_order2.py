"""The switch to second-order strain where the state is rough (Section 3,
after eq. itv; MHD_T_ORDER2) in the HIP library against the float64 oracle,
through the C ABI: right-hand sides, steps and the adjoint, on periodic and
wall-bounded boxes and anisotropic cells, in every tile shape and both
launch modes, alone and with quenching and the Smagorinsky viscosity.

The roughness limit of the mixed cases is put in the middle of a wide gap
between two of the state's sorted roughness values, far from every cell's
value, so that float64 rounding cannot move a cell across it; the float32
steps use a limit below every value (every cell rough), since there the
kernel's float32 logarithms decide the mask.

Tolerances as in the other parity tests: float64 <= 1e-12 relative L2 per
field, float32 steps <= 1e-5, adjoint <= 1e-10.
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle.stagger import AX_X, AX_Y, AX_Z
from paper_2405_02483_amd import inputs
from tests.helpers import grid_params, interior, rel_errors, to_cpu64

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
R2 = O.T_ORDER2


def _ctx(box, prm, dtype, **over):
    from paper_2405_02483_amd.lib import Context
    p = dict(prm)
    p.update(over)
    return Context(box, p, dtype=dtype)


def _rough(f, box, prm, seed):
    """The stratified states vary smoothly in ln rho and ln e_m (no cell is
    rough): add seeded 5% fluctuations of both."""
    rng = np.random.default_rng(seed)
    f = [a.copy() for a in f]
    f[0] = f[0] * np.exp(0.05 * rng.standard_normal(f[0].shape))
    f[4] = f[4] * np.exp(0.05 * rng.standard_normal(f[4].shape))
    return f, box, prm


def _case(name):
    if name == "turb_aniso":
        f, box, prm = inputs.turbulent(n=20, seed=36, kmax=3.0)
        f = [a[:18, :, :16].copy() for a in f]
        return f, dict(box, nx=16, ny=20, nz=18, Lx=1.1, Ly=0.8, Lz=1.35), prm
    if name == "turb_ragged":
        f, box, prm = inputs.turbulent(n=24, seed=32)
        f = [a[:, :22, :20].copy() for a in f]
        return f, dict(box, nx=20, ny=22, nz=24, Lx=20 / 24, Ly=22 / 24), prm
    if name == "strat":
        return _rough(*inputs.stratified(12, 10, 24, seed=33), seed=33)
    if name == "strat_aniso":
        f, box, prm = inputs.stratified(14, 10, 20, seed=38)
        return _rough(f, dict(box, Lx=box["Lx"] * 1.4, Ly=box["Ly"] * 0.7), prm, seed=38)
    if name == "min6":
        return inputs.turbulent(n=6, seed=34, kmax=2.0)
    raise KeyError(name)


CASES = ["turb_aniso", "turb_ragged", "strat", "strat_aniso", "min6"]


def _mid_gap_limit(f, box, frac=0.7):
    """A roughness limit with about `frac` of the cells below it, in the
    middle of the widest gap between neighbouring sorted values nearby."""
    g = O.Grid(**box)
    Ops = g.ops()
    ft = O.ghost_fill(to_cpu64(f), g)
    lr, le = torch.log(ft[0]), torch.log(ft[4] / ft[0])
    m = torch.zeros_like(lr)
    for a in (AX_X, AX_Y, AX_Z):
        for v in (lr, le):
            m = torch.maximum(m, Ops.d2abs(v, a))
    v = np.sort(m.numpy().ravel())
    n = len(v)
    lo, hi = int(0.6 * n), min(int(0.8 * n), n - 2)
    i = lo + int(np.argmax(v[lo + 1:hi + 2] - v[lo:hi + 1]))
    gap = v[i + 1] - v[i]
    assert gap > 1e-9 * v[i + 1]
    return 0.5 * (v[i] + v[i + 1])


def _variants(f, box):
    lim = _mid_gap_limit(f, box)
    return {
        "mixed": dict(terms=O.T_ALL | R2, d2_lim=lim),
        "mixed_c1": dict(terms=O.T_ALL | R2, d2_lim=lim, c1=-1.0 / 3.0),
        "all": dict(terms=O.T_ALL | R2, d2_lim=-1.0, c1=-1.0 / 3.0),
        "with_quench_smag": dict(terms=O.T_ALL | R2 | O.T_QUENCH | O.T_SMAG | O.T_MAX5, d2_lim=lim,
                                 c_smag=0.17, c1=-1.0 / 3.0),
    }


def _rhs_errs(f, box, prm, over, dtype=torch.float64, launch=None):
    ctx = _ctx(box, prm, dtype, **over)
    if launch:
        ctx.set_launch(*launch)
    F = ctx.box_view(ctx.rhs(ctx.upload([f])), 0)
    g, p = grid_params(box, prm, **over)
    want = O.rhs(to_cpu64(f), g, p)
    ctx.close()
    return rel_errors(F, want)


@pytest.mark.parametrize("variant", ["mixed", "mixed_c1", "all", "with_quench_smag"])
@pytest.mark.parametrize("case", CASES)
def test_rhs_parity_f64(case, variant):
    f, box, prm = _case(case)
    errs = _rhs_errs(f, box, prm, _variants(f, box)[variant])
    print(case, variant, ["%.2e" % e for e in errs])
    assert max(errs) < TOL64, errs


def test_switch_changes_the_rhs():
    f, box, prm = _case("turb_aniso")
    lim = _mid_gap_limit(f, box)
    out = []
    for over in (dict(terms=O.T_VISC), dict(terms=O.T_VISC | R2, d2_lim=lim)):
        ctx = _ctx(box, prm, torch.float64, **over)
        out.append([t.to("cpu", torch.float64) for t in ctx.box_view(ctx.rhs(ctx.upload([f])), 0)])
        ctx.close()
    errs = rel_errors(out[1], out[0])
    assert max(errs[1:5]) > 1e-3, errs


@pytest.mark.parametrize("tile", ["64x4", "32x8", "16x16", "16x8", "64x8", "32x16"])
@pytest.mark.parametrize("persistent", [False, True])
def test_every_launch_shape_f64(tile, persistent):
    f, box, prm = _case("strat_aniso")
    errs = _rhs_errs(f, box, prm, _variants(f, box)["with_quench_smag"], launch=(tile, persistent))
    assert max(errs) < TOL64, (tile, persistent, errs)


def test_launch_shapes_give_identical_bits_f32():
    from paper_2405_02483_amd.lib import TILES
    f, box, prm = _case("turb_ragged")
    ctx = _ctx(box, prm, torch.float32, **_variants(f, box)["mixed_c1"])
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
    """float64 with the mixed limit, float32 with every cell rough."""
    f, box, prm = _case(case)
    lim = _mid_gap_limit(f, box)
    for dtype, tol, over in ((torch.float64, TOL64, dict(terms=O.T_ALL | R2, d2_lim=lim, c1=-1.0 / 3.0)),
                             (torch.float32, 1e-5, dict(terms=O.T_ALL | R2, d2_lim=-1.0, c1=-1.0 / 3.0))):
        pr = dict(prm, **over)
        g, p = grid_params(box, pr)
        ft = O.ghost_fill(to_cpu64(f), g)
        dt = 0.5 * O.courant(ft, g, p)[0]
        want = O.step(ft, g, p, dt, 2)
        ctx = _ctx(box, pr, dtype)
        fd = ctx.upload([f])
        ctx.step(fd, dt, 2)
        got = ctx.box_view(fd, 0)
        if box.get("wall"):
            got, want = interior(got, box), interior(want, box)
        errs = rel_errors(got, want)
        assert max(errs) < tol, (dtype, errs)
        ctx.close()


@pytest.mark.parametrize("variant", ["mixed_c1", "all", "with_quench_smag"])
def test_step_adjoint_matches_oracle_f64(variant):
    f, box, prm = _case("turb_ragged")
    over = _variants(f, box)[variant]
    g, p = grid_params(box, prm, **over)
    ft = to_cpu64(f)
    dt = 0.5 * O.courant(ft, g, p)[0]
    rng = np.random.default_rng(41)
    gbar = [rng.standard_normal(a.shape) for a in f]
    ctx = _ctx(box, prm, torch.float64, **over)
    out = ctx.step_adjoint(ctx.upload([f]), dt, ctx.upload([gbar]))
    errs = rel_errors(ctx.box_view(out, 0), O.step_vjp(ft, g, p, dt, to_cpu64(gbar)))
    ctx.close()
    print(variant, ["%.2e" % e for e in errs])
    assert max(errs) < 1e-10, errs
