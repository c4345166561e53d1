"""Pins of the oracle's div B cleaning (Section 3, eq. clean1, eq. clean2)
by properties of the discrete operators alone: after cleaning the discrete
divergence vanishes; a discrete curl (B = curl A with the staggered up
derivatives of an edge potential, discretely solenoidal because operators
along different axes commute) is left unchanged; a discrete gradient
(B_a = ddadn(psi)) is removed entirely; a uniform field is kept; the
other fields are untouched; cleaning twice changes nothing more.  A wrong
operator symbol (a continuous k^2, a missing factor, the wrong half-cell
shift) breaks the first three.
"""
import pytest
import torch

import oracle as O

D = torch.float64


def _grid(shape, aniso):
    nx, ny, nz = shape
    if aniso:
        return O.Grid(nx, ny, nz, Lx=1.1, Ly=0.7, Lz=1.6)
    return O.Grid(nx, ny, nz)


def _rand(g, seed, k=4):
    gen = torch.Generator().manual_seed(seed)
    return [torch.randn(g.nzt, g.ny, g.nx, generator=gen, dtype=D) for _ in range(k)]


def _div(b, O_):
    return O_.ddxup(b[0]) + O_.ddyup(b[1]) + O_.ddzup(b[2])


def _curl(A, O_):
    ax, ay, az = A
    return (O_.ddyup(az) - O_.ddzup(ay), O_.ddzup(ax) - O_.ddxup(az), O_.ddxup(ay) - O_.ddyup(ax))


def _state(g, bx, by, bz, seed=1):
    r = _rand(g, seed + 100, 5)
    rho = 1.0 + 0.1 * r[0].abs()
    return (rho, r[1], r[2], r[3], 2.0 + r[4].abs(), bx, by, bz)


CASES = [((12, 10, 8), False), ((9, 14, 11), True), ((16, 16, 16), False)]


@pytest.mark.parametrize("shape,aniso", CASES)
def test_cleaned_field_is_discretely_solenoidal(shape, aniso):
    g = _grid(shape, aniso)
    Ops = g.ops()
    b = _rand(g, 2, 3)
    f = O.divb_clean(_state(g, *b), g)
    d0 = _div(b, Ops)
    d1 = _div(f[5:], Ops)
    assert float(d0.abs().max()) > 1.0
    assert float(d1.abs().max()) < 1e-12 * float(d0.abs().max())


@pytest.mark.parametrize("shape,aniso", CASES)
def test_curl_kept_gradient_removed_mean_kept(shape, aniso):
    g = _grid(shape, aniso)
    Ops = g.ops()
    A = _rand(g, 3, 3)
    psi = _rand(g, 4, 1)[0]
    curl = _curl(A, Ops)
    grad = (Ops.ddxdn(psi), Ops.ddydn(psi), Ops.ddzdn(psi))
    mean = (0.3, -0.7, 1.1)
    assert float(_div(curl, Ops).abs().max()) < 1e-10
    for what, b, want in (("curl", curl, curl), ("grad", grad, (0, 0, 0)),
                          ("all", [c + gr + m for c, gr, m in zip(curl, grad, mean)],
                           [c + m for c, m in zip(curl, mean)])):
        f = O.divb_clean(_state(g, *b), g)
        scale = max(float(torch.linalg.norm(x)) for x in b)
        for got, w in zip(f[5:], want):
            err = float(torch.linalg.norm(got - w)) if torch.is_tensor(w) else float(torch.linalg.norm(got - w))
            assert err < 1e-12 * scale, (what, err, scale)


def test_other_fields_untouched_and_idempotent():
    g = _grid((10, 12, 8), True)
    s = _state(g, *_rand(g, 5, 3))
    f1 = O.divb_clean(s, g)
    for a, b in zip(s[:5], f1[:5]):
        assert a is b or torch.equal(a, b)
    f2 = O.divb_clean(f1, g)
    for a, b in zip(f1[5:], f2[5:]):
        assert float(torch.linalg.norm(a - b)) < 1e-13 * float(torch.linalg.norm(a))


def test_walls_are_refused():
    g = O.Grid(8, 8, 8, wall=True, ngz=5)
    z = torch.zeros(g.nzt, 8, 8, dtype=D)
    with pytest.raises(ValueError):
        O.divb_clean((z + 1, z, z, z, z + 1, z, z, z), g)


def test_symbol_is_the_operator_on_a_mode():
    """The symbol used for the solve is what ddxup(ddxdn(.)) does to each
    Fourier mode of a periodic axis (checked by applying the operators)."""
    n = 12
    g = O.Grid(n, 6, 6, Lx=1.3)
    Ops = g.ops()
    K = O.derivative_symbol(n, g.dx)
    x = torch.arange(n, dtype=D)
    for m in range(n):
        f = torch.cos(2 * torch.pi * m * x / n + 0.3).view(1, 1, n).expand(6, 6, n).contiguous()
        lap = Ops.ddxup(Ops.ddxdn(f))
        assert torch.allclose(lap, -(K[m] ** 2) * f, rtol=0, atol=1e-11 * (1 + float(K[m] ** 2)))


@pytest.mark.parametrize("shape,aniso", CASES)
def test_cleaning_is_an_orthogonal_projection(shape, aniso):
    """On a periodic grid the down derivative is minus the transpose of the
    up derivative, so P = I - G (D G)^-1 D with D the divergence and G the
    gradient is symmetric: <P u, v> = <u, P v> for the sum over faces, and
    P u is orthogonal to every discrete gradient.  (Its adjoint is itself.)"""
    g = _grid(shape, aniso)
    Ops = g.ops()
    u, v = _rand(g, 5, 3), _rand(g, 6, 3)
    pu = O.divb_clean(_state(g, *u), g)[5:]
    pv = O.divb_clean(_state(g, *v), g)[5:]
    lhs = sum(float((a * b).sum()) for a, b in zip(pu, v))
    rhs = sum(float((a * b).sum()) for a, b in zip(u, pv))
    assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1.0)
    psi = _rand(g, 7, 1)[0]
    grad = (Ops.ddxdn(psi), Ops.ddydn(psi), Ops.ddzdn(psi))
    ip = sum(float((a * b).sum()) for a, b in zip(pu, grad))
    scale = (sum(float((a * a).sum()) for a in pu) * sum(float((a * a).sum()) for a in grad)) ** 0.5
    assert abs(ip) < 1e-12 * scale
