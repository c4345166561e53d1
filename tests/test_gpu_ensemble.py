"""Batched ensembles of uneven boxes: the persistent launch mode and the
autotuner (through the C ABI).  Every launch mode and tile shape must give
the same bits; an autotuned persistent ensemble must match the float64 oracle
box by box."""
import pytest
import torch

import oracle as O
from paper_2405_02483_amd import inputs
from tests.helpers import grid_params, rel_errors, to_cpu64

pytestmark = pytest.mark.gpu


def _ensemble(sizes, seed0=5000):
    cases = [inputs.turbulent(n=n, seed=seed0 + b, kmax=3.0) for b, n in enumerate(sizes)]
    return [c[0] for c in cases], [c[1] for c in cases], cases[0][2]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_persistent_mode_gives_identical_bits(dtype):
    from paper_2405_02483_amd.lib import Context, TILES
    fields, boxes, prm = _ensemble(inputs.ensemble_sizes(8, (6, 8, 12, 16), seed=5))
    ctx = Context(boxes, prm, dtype=dtype)
    ref = None
    for tile in TILES:
        for persistent in (0, 1):
            ctx.set_launch(tile, persistent)
            assert ctx.get_launch() == (tile, persistent)
            fd = ctx.upload(fields)
            ctx.step(fd, 0.0, 2)            # Courant dt on the device: exercises the partials
            dt = ctx.last_dt()
            if ref is None:
                ref = ([t.clone() for t in fd], dt)
            else:
                assert dt == ref[1], (tile, persistent)
                for a, b in zip(fd, ref[0]):
                    assert torch.equal(a, b), (tile, persistent)
    ctx.close()


def test_persistent_mode_walls_identical_bits():
    from paper_2405_02483_amd.lib import Context
    f, box, prm = inputs.stratified(12, 10, 24, seed=3)
    ctx = Context(box, prm, dtype=torch.float32)
    out = []
    for persistent in (0, 1):
        ctx.set_launch("32x8", persistent)
        fd = ctx.upload([f])
        ctx.step(fd, 0.0, 2)
        out.append(fd)
    for a, b in zip(*out):
        assert torch.equal(a, b)
    ctx.close()


def test_set_launch_rejects_bad_values():
    from paper_2405_02483_amd.lib import Context, MhdError, MHD_EINVAL, TILES
    f, box, prm = inputs.turbulent(n=8, seed=3, kmax=2.0)
    ctx = Context(box, prm, dtype=torch.float32)
    for tile, mode in ((len(TILES), 0), (-1, 0), (0, 2)):
        with pytest.raises(MhdError) as ei:
            ctx.set_launch(tile, mode)
        assert ei.value.code == MHD_EINVAL
    ctx.close()


def test_autotuned_persistent_ensemble_matches_oracle():
    from paper_2405_02483_amd.lib import Context, TILES
    sizes = inputs.ensemble_sizes(8, (6, 8, 10, 12), seed=5)
    fields, boxes, prm = _ensemble(sizes)
    ctx = Context(boxes, prm, dtype=torch.float32)
    fd = ctx.upload(fields)
    ms = ctx.autotune(fd, reps=2)
    assert len(ms) == 2 * len(TILES) and all(v > 0 for v in ms.values())
    # the shape of the fastest uniform launch; the mode and pass F's shape
    # may then change where that is faster still
    assert ctx.get_launch()[0] == min(ms, key=ms.get)[0]
    dt = 0.5 * min(O.courant(to_cpu64(f), *grid_params(b, prm))[0] for f, b in zip(fields, boxes))
    fd = ctx.upload(fields)
    ctx.step(fd, dt, 1)
    for b, (f, box) in enumerate(zip(fields, boxes)):
        g, p = grid_params(box, prm)
        want = O.step(to_cpu64(f), g, p, dt, 1)
        errs = rel_errors(ctx.box_view(fd, b), want)
        assert max(errs) < 1e-5, (b, sizes[b], errs)
    ctx.close()


@pytest.mark.parametrize("walls", [False, True])
def test_z_chunking_changes_no_bits(walls):
    """Small launches split z into more, shorter chunks (so that the device
    fills); a box stepped alone (three z-chunks) and the same box inside an
    ensemble large enough for one chunk per box must agree bit for bit."""
    from paper_2405_02483_amd.lib import Context
    if walls:
        f, box, prm = inputs.stratified(40, 40, 30, seed=7)      # 40 planes with ghosts
    else:
        f, box, prm = inputs.turbulent(n=40, seed=11, kmax=3.0)
    out = []
    for copies in (1, 110):                  # 10 items per box at 32x8; 1100 >= 4 per CU
        ctx = Context([box] * copies, prm, dtype=torch.float64)
        ctx.set_launch("32x8", 0)
        fd = ctx.upload([f] * copies)
        ctx.step(fd, 0.0, 2)
        out.append(([t.clone() for t in ctx.box_view(fd, 0)], ctx.last_dt()))
        ctx.close()
    assert out[0][1] == out[1][1]
    for a, b in zip(out[0][0], out[1][0]):
        assert torch.equal(a, b)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_final_pass_tile_gives_identical_bits(dtype):
    """Pass F in its own tile shape (its own work items and z-chunks) gives
    the same bits as the uniform launch; set_launch resets it."""
    from paper_2405_02483_amd.lib import Context, MhdError, MHD_EINVAL, TILES
    fields, boxes, prm = _ensemble(inputs.ensemble_sizes(6, (6, 10, 16), seed=6))
    ctx = Context(boxes, prm, dtype=dtype)
    ctx.set_launch("32x8", 0)
    assert ctx.get_final_tile() == "32x8"
    fd = ctx.upload(fields)
    ctx.step(fd, 0.0, 2)
    ref = ([t.clone() for t in fd], ctx.last_dt())
    for tile, ftile, persistent in (("16x16", "64x8", 0), ("64x8", "16x8", 1), ("32x8", "64x4", 1),
                                    ("32x16", "16x16", 0), ("16x8", "32x16", 1)):
        ctx.set_launch(tile, persistent)
        ctx.set_final_tile(ftile)
        assert ctx.get_launch() == (tile, persistent) and ctx.get_final_tile() == ftile
        fd = ctx.upload(fields)
        ctx.step(fd, 0.0, 2)
        assert ctx.last_dt() == ref[1]
        for a, b in zip(fd, ref[0]):
            assert torch.equal(a, b), (tile, ftile, persistent)
    ctx.set_launch("16x8", 0)
    assert ctx.get_final_tile() == "16x8"
    for bad in (-1, len(TILES)):
        with pytest.raises(MhdError) as ei:
            ctx.set_final_tile(bad)
        assert ei.value.code == MHD_EINVAL
    ctx.close()


def test_benchmark_ensemble_boxes_match_oracle():
    """The bench's 96-box float32 ensemble (24 each of 48^3, 64^3, 80^3,
    96^3, turbulent, seeds 5000 + b) in its autotuned launch: one RK step
    with the Courant dt taken on the device, then the first 48^3 and the
    first 96^3 box against the oracle's step of that box alone (<= 1e-5
    relative L2 per field)."""
    import math
    from paper_2405_02483_amd.lib import Context
    cases, prm = inputs.ensemble()
    sizes = [c[1]["nx"] for c in cases]
    ctx = Context([c[1] for c in cases], prm, dtype=torch.float32)
    fd = ctx.upload([c[0] for c in cases])
    ctx.autotune(fd, reps=2)
    print("launch", ctx.get_launch(), "pass F", ctx.get_final_tile())
    fd = ctx.upload([c[0] for c in cases])
    ctx.step(fd, 0.0, 1)
    dt = ctx.last_dt()
    want_dt = min(O.courant(to_cpu64(f), *grid_params(b, prm))[0] for f, b in cases)
    assert math.isclose(dt, want_dt, rel_tol=1e-6), (dt, want_dt)
    for n in (48, 96):
        b = sizes.index(n)
        f, box = cases[b]
        g, p = grid_params(box, prm)
        want = O.step(to_cpu64(f), g, p, dt, 1)
        errs = rel_errors(ctx.box_view(fd, b), want)
        print(n, b, ["%.1e" % e for e in errs])
        assert max(errs) < 1e-5, (n, b, errs)
    ctx.close()
