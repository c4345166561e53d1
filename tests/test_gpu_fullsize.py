"""Parity at the benchmark's full size: the 512^3 stratified box (walls in z,
5 ghost planes per side) in float32, with the stage kernels in the launch
configuration bench.py times (autotuned on the same state), in the library
default and in the persistent 16x16 configuration.

The oracle cannot hold the whole box, so it checks sampled columns.  The
right-hand side at a cell depends on cells at most 11 cells away along x and
y (measured with the oracle: a perturbation of one cell changes F no further
out), 14 near closed walls (the ghost momenta interpolate the density along
x and y first), and one RK step on at most 3 x 14.  A full-height window of the state,
periodic in x and y with width 2 m + w, therefore gives the oracle's exact
result on its central w x w columns when m covers that radius.  Properties
that hold at any size (mass conservation with closed walls, div B at
rounding level) are checked on the whole box.

In hydrostatic balance the momentum right-hand side is a small residual of
the pressure gradient and gravity, so float32 errors of F are measured
against the size of the terms being summed: per field, the error norm over
the sum of the norms of that field's term groups (the oracle run with one
group of terms at a time), at most 1e-4.  The state after one step is held to
the stated float32 tolerance, 1e-5 relative L2.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2405_02483_amd import inputs
from tests.helpers import grid_params, rel_errors

TERM_GROUPS = (O.T_CONT, O.T_ADV, O.T_PRES, O.T_VISC, O.T_LORENTZ, O.T_INDUCT, O.T_RESIST,
               O.T_EDIFF, O.T_GRAV)

pytestmark = pytest.mark.gpu

N = 512
RHS_MARGIN = 16
STEP_MARGIN = 44


@pytest.fixture(scope="module")
def state():
    f, box, prm = inputs.stratified(N, N, N, seed=3)
    return f, box, prm


def _window(f, box, x0, y0, width):
    ix = (np.arange(width) + x0) % box["nx"]
    iy = (np.arange(width) + y0) % box["ny"]
    sub = [torch.from_numpy(np.ascontiguousarray(np.asarray(a)[:, iy][:, :, ix])).to(torch.float64)
           for a in f]
    wbox = dict(box, nx=width, ny=width, Lx=box["Lx"] * width / box["nx"],
                Ly=box["Ly"] * width / box["ny"])
    return sub, wbox


def _centre(a, margin):
    return a[:, margin:-margin, margin:-margin]


def _term_scale(sub, wbox, prm, crop):
    """Per field, the sum of the norms of what its right-hand side adds up:
    each term group (the oracle with one group on), and for rho the three
    derivatives of -div p separately (they cancel for a solenoidal p)."""
    scale = [0.0] * 8
    for t in TERM_GROUPS:
        gt, pt = grid_params(wbox, prm, terms=t)
        for v, a in enumerate(O.rhs(tuple(sub), gt, pt)):
            if v != 0:
                scale[v] += float(torch.linalg.norm(crop(a)))
    g, _ = grid_params(wbox, prm)
    Op = g.ops()
    for q in (Op.ddxup(sub[1]), Op.ddyup(sub[2]), Op.ddzup(sub[3])):
        scale[0] += float(torch.linalg.norm(crop(q)))
    return scale


def _scaled_errors(got, want, scale):
    return [float(torch.linalg.norm(a - b)) / max(sc, 1e-300) for a, b, sc in zip(got, want, scale)]


def _windows(seed, count, width):
    rng = np.random.default_rng(seed)
    return [tuple(int(v) for v in rng.integers(0, N, 2)) for _ in range(count)]


@pytest.mark.parametrize("launch", ["autotuned", None, ("16x16", 1), ("32x16", 0)])
def test_rhs_sampled_columns_512(state, launch):
    from paper_2405_02483_amd.lib import Context
    f, box, prm = state
    ctx = Context(box, prm, dtype=torch.float32)
    fd = ctx.upload([f])
    if launch == "autotuned":
        ctx.autotune(fd, reps=2)                 # as bench.py
        print("launch", ctx.get_launch(), "pass F", ctx.get_final_tile())
    elif launch:
        ctx.set_launch(*launch)
    F = [t.view(-1) for t in ctx.box_view(ctx.rhs(fd), 0)]
    nzt = N + 2 * box["ngz"]
    width = 2 * RHS_MARGIN + 8
    for x0, y0 in _windows(51, 4, width):
        sub, wbox = _window(f, box, x0, y0, width)
        g, p = grid_params(wbox, prm)
        want = [_centre(a, RHS_MARGIN) for a in O.rhs(tuple(sub), g, p)]
        scale = _term_scale(sub, wbox, prm, lambda a: _centre(a, RHS_MARGIN))
        ix = torch.from_numpy((np.arange(RHS_MARGIN, width - RHS_MARGIN) + x0) % N)
        iy = torch.from_numpy((np.arange(RHS_MARGIN, width - RHS_MARGIN) + y0) % N)
        got = [t.view(nzt, N, N)[:, iy.cuda()][:, :, ix.cuda()].cpu().double() for t in F]
        errs = _scaled_errors(got, want, scale)
        print((x0, y0), ["%.1e" % e for e in errs], "plain", ["%.1e" % e for e in rel_errors(got, want)])
        assert max(errs) < 1e-4, ((x0, y0), errs)
    ctx.close()


def test_step_sampled_columns_and_invariants_512(state):
    from paper_2405_02483_amd.lib import Context
    f, box, prm = state
    ctx = Context(box, prm, dtype=torch.float32)
    fd = ctx.upload([f])
    ctx.autotune(fd, reps=2)                     # as bench.py (fills the ghosts of fd)
    s0 = ctx.reductions(fd)
    ctx.step(fd, 0.0, 1)                       # as bench.py: Courant dt on the device
    dt = ctx.last_dt()
    assert math.isclose(dt, s0["dt"], rel_tol=1e-6), (dt, s0["dt"])
    s1 = ctx.reductions(fd)
    assert abs(s1["mass"] - s0["mass"]) <= 1e-6 * s0["mass"]
    assert s1["divb_max"] * (1.0 / N) <= 1e-5 * s1["bmax"]
    nzt = N + 2 * box["ngz"]
    got_all = [t.view(nzt, N, N) for t in ctx.box_view(fd, 0)]
    width = 2 * STEP_MARGIN + 16
    g0, g1 = box["ngz"], box["ngz"] + N
    for x0, y0 in _windows(52, 2, width):
        sub, wbox = _window(f, box, x0, y0, width)
        g, p = grid_params(wbox, prm)
        want = [_centre(a, STEP_MARGIN)[g0:g1] for a in O.step(tuple(sub), g, p, dt, 1)]
        ix = torch.from_numpy((np.arange(STEP_MARGIN, width - STEP_MARGIN) + x0) % N).cuda()
        iy = torch.from_numpy((np.arange(STEP_MARGIN, width - STEP_MARGIN) + y0) % N).cuda()
        got = [t[g0:g1][:, iy][:, :, ix].cpu() for t in got_all]
        errs = rel_errors(got, want)
        print((x0, y0), ["%.1e" % e for e in errs])
        assert max(errs) < 1e-5, ((x0, y0), errs)
    ctx.close()


# ---------------------------------------------------------------------------
# The 256^3 periodic turbulent box (seed 2) in float32 and float64: one
# right-hand side and one RK step, checked on cubic windows (periodic in all
# three axes, so the window is cut along z too).  The momenta of this state
# are solenoidal, so -div p is a residual of derivatives about 10^4 times
# larger; right-hand sides are measured against the size of what is summed
# (as for the stratified box), the stepped state by plain relative L2.

M2 = 256


@pytest.fixture(scope="module")
def turb256():
    return inputs.turbulent(n=M2, seed=2)


def _cube(f, box, c, width):
    idx = [(np.arange(width) + c[a]) % M2 for a in range(3)]
    sub = [torch.from_numpy(np.ascontiguousarray(np.asarray(a)[idx[2]][:, idx[1]][:, :, idx[0]]))
           .to(torch.float64) for a in f]
    h = box["Lx"] / box["nx"]
    wbox = dict(box, nx=width, ny=width, nz=width, Lx=h * width, Ly=h * width, Lz=h * width)
    return sub, wbox, idx


def _gather(t, idx, margin, width):
    sel = [torch.from_numpy(i[margin:width - margin]).cuda() for i in idx]
    return t.view(M2, M2, M2)[sel[2]][:, sel[1]][:, :, sel[0]].cpu().double()


def _core(a, m):
    return a[m:-m, m:-m, m:-m]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_turbulent_256_rhs_and_step_sampled(turb256, dtype):
    from paper_2405_02483_amd.lib import Context
    f, box, prm = turb256
    ctx = Context(box, prm, dtype=dtype)
    fd = ctx.upload([f])
    F = ctx.rhs(fd)
    tol_rhs, tol_step = (1e-4, 1e-5) if dtype == torch.float32 else (1e-12, 1e-12)
    rng = np.random.default_rng(53)
    width = 2 * RHS_MARGIN + 8
    for _ in range(3):
        c = [int(v) for v in rng.integers(0, M2, 3)]
        sub, wbox, idx = _cube(f, box, c, width)
        g, p = grid_params(wbox, prm)
        want = [_core(a, RHS_MARGIN) for a in O.rhs(tuple(sub), g, p)]
        got = [_gather(t, idx, RHS_MARGIN, width) for t in F]
        errs = _scaled_errors(got, want, _term_scale(sub, wbox, prm, lambda a: _core(a, RHS_MARGIN)))
        print("rhs", dtype, c, ["%.1e" % e for e in errs])
        assert max(errs) < tol_rhs, (c, errs)
    ctx.step(fd, 0.0, 1)                       # Courant dt on the device
    dt = ctx.last_dt()
    width = 2 * 36 + 12                        # one step reaches 3 x 11 cells
    c = [int(v) for v in rng.integers(0, M2, 3)]
    sub, wbox, idx = _cube(f, box, c, width)
    g, p = grid_params(wbox, prm)
    want = [_core(a, 36) for a in O.step(tuple(sub), g, p, dt, 1)]
    got = [_gather(t, idx, 36, width) for t in fd]
    errs = rel_errors(got, want)
    print("step", dtype, c, ["%.1e" % e for e in errs])
    assert max(errs) < tol_step, (c, errs)
    ctx.close()


# ---------------------------------------------------------------------------
# The 512^3 isothermal atmosphere at rest (no velocity noise, uniform
# vertical field) in float64: hydrostatic balance holds to truncation, which
# at this resolution is below rounding, so the state must stay at rest.  The
# state is horizontally uniform, so every column of the right-hand side must
# be the same, and a 6 x 6 x 512 oracle box (periodic in x and y) gives that
# column exactly.

def test_static_atmosphere_512_float64():
    from paper_2405_02483_amd.lib import Context
    f, box, prm = inputs.stratified(N, N, N, seed=3, noise=0.0)
    ctx = Context(box, prm, dtype=torch.float64)
    fd = ctx.upload([f])
    nzt = N + 2 * box["ngz"]
    F = [t.view(nzt, N, N) for t in ctx.box_view(ctx.rhs(fd), 0)]
    for v, t in enumerate(F):
        assert torch.equal(t, t[:, :1, :1].expand_as(t)), v      # identical columns
    # the oracle on a 6 x 6 box of the same columns
    sub = [torch.from_numpy(np.ascontiguousarray(np.asarray(a)[:, :6, :6])).to(torch.float64) for a in f]
    wbox = dict(box, nx=6, ny=6, Lx=box["Lx"] * 6 / N, Ly=box["Ly"] * 6 / N)
    g, p = grid_params(wbox, prm)
    want = O.rhs(tuple(sub), g, p)
    # the momentum residual cancels the pressure gradient and gravity (size
    # g rho, about 4): compare absolutely against that scale
    scale = float(prm["gz"]) * float(torch.as_tensor(np.asarray(f[0])).max())
    for v in range(8):
        err = float((F[v][:, 0, 0].cpu() - want[v][:, 0, 0]).abs().max())
        assert err <= 1e-12 * scale, (v, err, scale)
    # ten Courant steps: the gas stays at rest to rounding
    s0 = ctx.reductions(fd)
    ctx.step(fd, 0.0, 10)
    s1 = ctx.reductions(fd)
    cs = math.sqrt(prm["gamma"])                     # isothermal: P = rho
    print("max |u| / c_s after 10 steps: %.2e" % (s1["umax"] / cs))
    assert s1["umax"] / cs <= 1e-10
    assert abs(s1["mass"] - s0["mass"]) <= 1e-13 * s0["mass"]
    ctx.close()
