"""Pins of the oracle's staggered operators against what the paper and the
mathematics fix (not against the oracle itself).

* printed coefficients (eq. derivcoef, eq. interpcoef) via tests/golden;
* closed forms on sinusoids, which fix both the coefficients and the
  staggering (a wrong index shift changes the phase);
* sixth-order convergence of the derivative;
* exactness on polynomials (degree <= 6 for the derivative, <= 5 for the
  interpolation: the paper's "fifth order" interpolation), and the reduced
  orders next to the ends of a wall-bounded axis;
* the max-then-mean spreading of the viscosity on an impulse (Section 6.1.1).
"""
import json
import math
import os
from fractions import Fraction

import pytest
import torch

import oracle as O
from oracle.stagger import AX_X, AX_Y, AX_Z

D = torch.float64


def _frac(s):
    return float(Fraction(s))


def test_coefficients_match_printed_values(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "paper_constants.json")))
    a, b, c = O.DERIV6
    assert a == _frac(g["deriv6"]["a"])
    assert b == _frac(g["deriv6"]["b"])
    assert c == _frac(g["deriv6"]["c"])
    a, b, c = O.INTERP6
    assert a == _frac(g["interp6"]["a"])
    assert b == _frac(g["interp6"]["b"])
    assert c == _frac(g["interp6"]["c"])


def _grid_axis(n, L, axis, shape, face):
    h = L / n
    x = (torch.arange(n, dtype=D) + (0.0 if face else 0.5)) * h
    s = [1, 1, 1]
    s[axis] = n
    return x.view(s).expand(shape), h


SYM = {  # symbol of each operator on exp(i k x): (kind, factor)
    "i": lambda k, h: 2.0 * sum(w * math.cos((2 * p - 1) * k * h / 2)
                                for p, w in enumerate(O.INTERP6, 1)),
    "d": lambda k, h: (2.0 / h) * sum(w * math.sin((2 * p - 1) * k * h / 2)
                                      for p, w in enumerate(O.DERIV6, 1)),
}


@pytest.mark.parametrize("axis", [AX_X, AX_Y, AX_Z])
@pytest.mark.parametrize("fam", ["i", "d"])
@pytest.mark.parametrize("form", ["dn", "up"])
def test_closed_form_on_sinusoid(axis, fam, form):
    """f = sin(k x + phi) sampled where the operator's input lives; result
    must equal S(k) * {sin|cos}(k x_out + phi) at the output location, with
    S the operator's symbol written from the trigonometric identity."""
    n, L = 24, 1.3
    shape = [10, 11, 12]
    shape[axis] = n
    shape = tuple(shape)
    ops = O.Ops(L / n if axis == AX_X else 0.1, L / n if axis == AX_Y else 0.1,
                L / n if axis == AX_Z else 0.1)
    for m in (1, 3, 7):
        k = 2 * math.pi * m / L
        phi = 0.3 * m
        # dn: input at centres, output at faces; up: input at faces, output at centres
        xin, h = _grid_axis(n, L, axis, shape, face=(form == "up"))
        xout, _ = _grid_axis(n, L, axis, shape, face=(form == "dn"))
        f = torch.sin(k * xin + phi)
        got = ops.stencil(f, axis, fam, form)
        S = SYM[fam](k, h)
        want = S * (torch.sin(k * xout + phi) if fam == "i" else torch.cos(k * xout + phi))
        assert torch.allclose(got, want, rtol=0, atol=1e-13 * max(1.0, abs(S))), (m, fam, form)


def test_sixth_order_convergence():
    errs = []
    for n in (16, 32, 64):
        h = 1.0 / n
        ops = O.Ops(h, h, h)
        xc = (torch.arange(n, dtype=D) + 0.5) * h
        f = torch.sin(2 * math.pi * xc).view(1, 1, n).expand(2, 2, n)
        d = ops.ddxdn(f)
        xf = torch.arange(n, dtype=D) * h
        exact = 2 * math.pi * torch.cos(2 * math.pi * xf)
        errs.append(float((d[0, 0] - exact).abs().max()))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 55 < r1 < 70 and 55 < r2 < 70, errs
    # interpolation: also sixth order
    errs = []
    for n in (16, 32, 64):
        h = 1.0 / n
        ops = O.Ops(h, h, h)
        xc = (torch.arange(n, dtype=D) + 0.5) * h
        f = torch.sin(2 * math.pi * xc).view(1, 1, n).expand(2, 2, n)
        v = ops.xdn(f)
        xf = torch.arange(n, dtype=D) * h
        errs.append(float((v[0, 0] - torch.sin(2 * math.pi * xf)).abs().max()))
    assert 55 < errs[0] / errs[1] < 70 and 55 < errs[1] / errs[2] < 70, errs


def _poly_z(coefs, z):
    return sum(c * z ** p for p, c in enumerate(coefs))


def _dpoly_z(coefs, z):
    return sum(p * c * z ** (p - 1) for p, c in enumerate(coefs) if p > 0)


@pytest.mark.parametrize("form", ["dn", "up"])
def test_wall_axis_polynomial_exactness(form):
    """Wall-bounded z: sixth-order interior exact for degree 6 (derivative)
    and 5 (interpolation); 4th-order planes for degree 4 / 3; 2nd-order planes
    for degree 2 / 1; the one unreachable end plane copies its neighbour."""
    n, h = 20, 0.1
    ops = O.Ops(0.1, 0.1, h, wall_z=True)
    zc = (torch.arange(n, dtype=D) + 0.5) * h
    zf = torch.arange(n, dtype=D) * h
    zin = zc if form == "dn" else zf
    zout = zf if form == "dn" else zc          # same index, half a cell away
    off = 0 if form == "dn" else 1

    def order_at(k):
        c = k + off
        for o in (6, 4, 2):
            q = o // 2
            if c - q >= 0 and c + q - 1 <= n - 1:
                return o
        return None

    orders = [order_at(k) for k in range(n)]
    assert orders.count(None) == 1 and orders.count(4) == 2 and orders.count(2) == 2
    torch.manual_seed(0)
    for fam, degmax in (("d", {6: 6, 4: 4, 2: 2}), ("i", {6: 5, 4: 3, 2: 1})):
        for o in (6, 4, 2):
            coefs = torch.randn(degmax[o] + 1, dtype=D).tolist()
            f = _poly_z(coefs, zin).view(n, 1, 1).expand(n, 3, 3).contiguous()
            got = ops.stencil(f, AX_Z, fam, form)[:, 0, 0]
            want = (_dpoly_z if fam == "d" else _poly_z)(coefs, zout)
            for k, ok in enumerate(orders):
                if ok is None:
                    assert got[k] == got[1 if k == 0 else n - 2]
                elif ok >= o:
                    assert abs(float(got[k] - want[k])) < 1e-9 * (1 + abs(float(want[k]))), (fam, o, k)


def test_operator_transposes():
    """Summation by parts on a periodic axis: <ddup f, g> = -<f, dddn g> and
    <up f, g> = <f, dn g>; the adjoint relations the discrete adjoint uses."""
    torch.manual_seed(1)
    ops = O.Ops(0.1, 0.2, 0.3)
    f = torch.randn(8, 9, 10, dtype=D)
    g = torch.randn(8, 9, 10, dtype=D)
    for ax in (AX_X, AX_Y, AX_Z):
        a = (ops.stencil(f, ax, "d", "up") * g).sum()
        b = -(f * ops.stencil(g, ax, "d", "dn")).sum()
        assert abs(float(a - b)) < 1e-12 * float(f.abs().sum() * g.abs().max())
        a = (ops.stencil(f, ax, "i", "up") * g).sum()
        b = (f * ops.stencil(g, ax, "i", "dn")).sum()
        assert abs(float(a - b)) < 1e-12 * float(f.abs().sum() * g.abs().max())


def test_max_then_mean_spreading_of_impulse():
    """Section 6.1.1: maximum over three adjacent cells, then a three-cell
    average, in each direction.  An isolated peak v on a zero background gives
    v * w(dx) w(dy) w(dz) with w = (1/3, 2/3, 1, 2/3, 1/3) over offsets -2..2."""
    n = 9
    ops = O.Ops(0.1, 0.1, 0.1)
    f = torch.zeros(n, n, n, dtype=D)
    f[4, 4, 4] = 3.0
    m = ops.max3(ops.max3(ops.max3(f, AX_X), AX_Y), AX_Z)
    s = ops.mean3(ops.mean3(ops.mean3(m, AX_X), AX_Y), AX_Z)
    w = torch.zeros(n, dtype=D)
    w[2:7] = torch.tensor([1 / 3, 2 / 3, 1.0, 2 / 3, 1 / 3], dtype=D)
    want = 3.0 * w.view(n, 1, 1) * w.view(1, n, 1) * w.view(1, 1, n)
    assert torch.allclose(s, want, atol=1e-15)


def test_max3_tie_selects_first():
    """The tie rule the adjoint depends on: first maximal element."""
    a = torch.tensor([2.0, 2.0, 2.0], dtype=D, requires_grad=True)
    m = torch.stack([a[0:1], a[1:2], a[2:3]]).max(dim=0).values
    m.sum().backward()
    assert a.grad.tolist() == [1.0, 0.0, 0.0]
