"""mhd_rhs_noalloc, the variant of mhd_rhs that allocates nothing (its
per-call scratch lives in the library's static device array), against
mhd_rhs through the C ABI: bit for bit on two calls in a row, the second
with a smaller box, in both precisions and with the optional terms whose
per-plane tables also live in the scratch; and the refusal of a box too
large for the array."""
import numpy as np
import pytest
import torch

from paper_2405_02483_amd import inputs

pytestmark = pytest.mark.gpu


def _big():
    # walled box with the plane-mean terms (their tables use the scratch too)
    f, box, prm = inputs.stratified(20, 18, 24, seed=41)
    from paper_2405_02483_amd.lib import T_ALL, T_EDIFFAV, T_LNP, T_COOL
    return f, box, dict(prm, terms=T_ALL | T_EDIFFAV | T_LNP | T_COOL, e_cool=1.3, t_cool=0.4)


def _small():
    f, box, prm = inputs.turbulent(n=10, seed=42, kmax=2.0)
    f = [np.ascontiguousarray(a[:9, :, :]) for a in f]
    return f, dict(box, nz=9, Lz=0.9), prm


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_matches_rhs_on_two_calls(dtype):
    from paper_2405_02483_amd.lib import Context
    for (f, box, prm), (tile, pers) in ((_big(), ("64x8", 1)), (_small(), ("16x8", 0))):
        ctx = Context(box, prm, dtype=dtype)
        ctx.set_launch(tile, pers)
        fd = ctx.upload([f])
        want = ctx.rhs(fd)
        got = ctx.rhs_noalloc(fd, ctx.empty())
        torch.cuda.synchronize()
        for v, (a, b) in enumerate(zip(got, want)):
            assert torch.equal(a, b), (dtype, box["nx"], v, float((a - b).abs().max()))
        ctx.close()


def test_noalloc_refuses_a_box_above_the_limit():
    """96^3 float32 needs 34 x 96^3 x 4 bytes (120 MB) of workspace, above
    the 64 MiB array: MHD_EINVAL with the sizes in the message, and nothing
    written."""
    from paper_2405_02483_amd.lib import Context, MhdError, MHD_EINVAL
    f, box, prm = inputs.turbulent(n=96, seed=43, kmax=2.0)
    ctx = Context(box, prm, dtype=torch.float32)
    fd = ctx.upload([f])
    out = ctx.empty()
    for t in out:
        t.fill_(7.0)
    with pytest.raises(MhdError) as ei:
        ctx.rhs_noalloc(fd, out)
    assert ei.value.code == MHD_EINVAL and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert all(bool((t == 7.0).all()) for t in out)
    ctx.close()
