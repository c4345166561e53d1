"""Staggered 1-D operators of the Stagger Code (paper Section 4, "Space
Operations": eq. deriv, eq. derivcoef, eq. interp, eq. interpcoef).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Arrays are float64 torch tensors indexed ``[z, y, x]`` (axis 0 = z, 1 = y,
2 = x).  Storage convention (Section 4.1, "Centering"): density, energy and
pressure sit at cell centres; momenta, velocities and magnetic field sit on
the cell face at the *lower* index side, so element ``i`` of a face array lives
at position ``i - 1/2`` in cell-index units.  Edge quantities (electric field,
current, off-diagonal stress) sit on the lower-index edges.

Two families, each in an "up" and a "down" form (Section 4.2 and 4.3 say that
similar formulas are used for each direction and for downward operators):

* ``dn`` / ``ddn``:  value at ``i - 1/2`` from samples at integer positions
  (centre -> lower face);
* ``up`` / ``dup``:  value at ``i + 1/2`` from samples at ``j`` (relative), used
  to go from a lower face back to the centre of the same index.

With ``c`` the index of the sample just above the output point (``c = i`` for
the down form, ``c = i + 1`` for the up form), pair ``p`` (p = 1, 2, 3) is the
symmetric pair ``(c - p, c + p - 1)`` and

    interpolation:  sum_p w_p * (f[c+p-1] + f[c-p])          (eq. interp)
    derivative:     sum_p d_p * (f[c+p-1] - f[c-p]) / h      (eq. deriv)

Periodic axes wrap (Section 4.2: values beyond the boundary are taken from
the opposite side).  A wall-bounded z axis (ghost zones, Section 10) uses the
same formula where all six samples exist; nearer the array ends the order
drops to the widest centred stencil that fits (4th order, then 2nd order),
and the single end value that no stencil reaches copies its neighbour.  This
is the reading of Section 10's remark that every operation destroys the
outermost valid ghost zone.
"""
from fractions import Fraction

import torch

__all__ = [
    "DERIV6", "INTERP6", "DERIV4", "INTERP4", "DERIV2", "INTERP2",
    "AX_X", "AX_Y", "AX_Z", "Ops",
]

# ---------------------------------------------------------------------------
# Coefficients, computed exactly from the paper's own expressions and rounded
# once to float64.
# eq. derivcoef:  c = (-1 + (3^5-3)/(3^3-3)) / (5^5 - 5 - 5(3^5-3)),
#                 b = (-1 - 120 c)/24,  a = 1 - 3b - 5c
_c = (Fraction(-1) + Fraction(3**5 - 3, 3**3 - 3)) / Fraction(5**5 - 5 - 5 * (3**5 - 3))
_b = (Fraction(-1) - 120 * _c) / 24
_a = 1 - 3 * _b - 5 * _c
DERIV6 = (float(_a), float(_b), float(_c))          # 75/64, -25/384, 3/640
# eq. interpcoef:  c = 3/256, b = -25/256, a = 1/2 - b - c
_ic = Fraction(3, 256)
_ib = Fraction(-25, 256)
_ia = Fraction(1, 2) - _ib - _ic
INTERP6 = (float(_ia), float(_ib), float(_ic))      # 150/256, -25/256, 3/256
# Reduced orders used only next to the ends of a wall-bounded axis: the
# standard centred staggered 4th-order (27/24, -1/24) and 2nd-order stencils.
DERIV4 = (9.0 / 8.0, -1.0 / 24.0)
INTERP4 = (9.0 / 16.0, -1.0 / 16.0)
DERIV2 = (1.0,)
INTERP2 = (0.5,)

_COEF = {
    ("i", 6): INTERP6, ("i", 4): INTERP4, ("i", 2): INTERP2,
    ("d", 6): DERIV6, ("d", 4): DERIV4, ("d", 2): DERIV2,
}

AX_Z, AX_Y, AX_X = 0, 1, 2


def _shift(f, m, axis):
    """g[i] = f[i + m] along ``axis`` with periodic wrap."""
    return torch.roll(f, shifts=-m, dims=axis)


def _pair_formula(get, fam, order, h):
    """Evaluate the centred staggered stencil of ``order`` from pair samples.

    ``get(p)`` returns the tuple (f[c+p-1], f[c-p]) for pair p.
    """
    coef = _COEF[(fam, order)]
    acc = None
    for p, w in enumerate(coef, start=1):
        hi, lo = get(p)
        term = w * (hi + lo) if fam == "i" else w * (hi - lo)
        acc = term if acc is None else acc + term
    if fam == "d":
        acc = acc / h
    return acc


class Ops:
    """The paper's operators on one box.

    ``wall_z``: if true, axis 0 (z) is not periodic and uses the reduced-order
    end treatment described in the module docstring; x and y are always
    periodic (Section 10).
    ``h``: grid spacings (dx, dy, dz).
    ``jz``: a stretched z axis (walls only): (Jc, Jf), the Jacobians of each
    plane's centre and face (Section 4.2: derivatives in index space times
    the Jacobian at the derivative's centre); an up derivative's output sits
    at a centre, a down derivative's on a face.
    """

    def __init__(self, dx, dy, dz, wall_z=False, jz=None):
        self.h = {AX_X: dx, AX_Y: dy, AX_Z: dz}
        self.wall_z = wall_z
        self.jz = jz

    # -- generic -----------------------------------------------------------
    def stencil(self, f, axis, fam, form, order=6):
        """fam: 'i' (interpolation) or 'd' (derivative); form: 'dn' or 'up';
        order: 6, or 2 for the second-order stencil (the strain where the
        state is rough, the switch after eq. itv)."""
        h = self.h[axis]
        if axis == AX_Z and self.wall_z:
            jac = None
            if self.jz is not None and fam == "d":
                jac = self.jz[0] if form == "up" else self.jz[1]
            return self._wall_stencil(f, fam, form, h, order, jac)
        off = 0 if form == "dn" else 1      # c = i + off

        def get(p):
            return _shift(f, off + p - 1, axis), _shift(f, off - p, axis)
        return _pair_formula(get, fam, order, h)

    def _wall_stencil(self, f, fam, form, h, top=6, jac=None):
        n = f.shape[0]
        off = 0 if form == "dn" else 1
        planes = [None] * n
        for k in range(n):
            c = k + off
            order = None
            for o in (6, 4, 2):
                if o > top:
                    continue
                q = o // 2
                if c - q >= 0 and c + q - 1 <= n - 1:
                    order = o
                    break
            if order is None:
                continue

            def get(p, c=c):
                return f[c + p - 1], f[c - p]
            if jac is None:
                planes[k] = _pair_formula(get, fam, order, h)
            else:     # index space, times this output's Jacobian
                planes[k] = _pair_formula(get, fam, order, 1.0) * jac[k]
        # the one end value no centred stencil reaches copies its neighbour
        if planes[0] is None:
            planes[0] = planes[1]
        if planes[n - 1] is None:
            planes[n - 1] = planes[n - 2]
        return torch.stack(planes)

    # -- named operators (the Stagger Code's xdn / xup / ddxdn / ddxup ...) --
    def xdn(self, f): return self.stencil(f, AX_X, "i", "dn")
    def ydn(self, f): return self.stencil(f, AX_Y, "i", "dn")
    def zdn(self, f): return self.stencil(f, AX_Z, "i", "dn")
    def xup(self, f): return self.stencil(f, AX_X, "i", "up")
    def yup(self, f): return self.stencil(f, AX_Y, "i", "up")
    def zup(self, f): return self.stencil(f, AX_Z, "i", "up")
    def ddxdn(self, f): return self.stencil(f, AX_X, "d", "dn")
    def ddydn(self, f): return self.stencil(f, AX_Y, "d", "dn")
    def ddzdn(self, f): return self.stencil(f, AX_Z, "d", "dn")
    def ddxup(self, f): return self.stencil(f, AX_X, "d", "up")
    def ddyup(self, f): return self.stencil(f, AX_Y, "d", "up")
    def ddzup(self, f): return self.stencil(f, AX_Z, "d", "up")

    # -- spreading and smoothing of the viscosity (Section 6.1.1) -----------
    def max3(self, f, axis):
        """Maximum over the three adjacent cells i-1, i, i+1.  In a tie the
        first maximal element in the order (i-1, i, i+1) is the selected one
        (this fixes the subgradient the adjoint uses)."""
        if axis == AX_Z and self.wall_z:
            n = f.shape[0]
            planes = []
            for k in range(n):
                cand = [f[j] for j in (k - 1, k, k + 1) if 0 <= j < n]
                planes.append(torch.stack(cand).max(dim=0).values)
            return torch.stack(planes)
        lo, hi = _shift(f, -1, axis), _shift(f, 1, axis)
        return torch.stack([lo, f, hi]).max(dim=0).values

    def max5(self, f, axis):
        """Maximum over the five adjacent cells i-2 .. i+2 (over the available
        ones at the ends of a wall-bounded axis): the three-cell maximum
        applied twice, which also fixes the adjoint's choice in a tie."""
        return self.max3(self.max3(f, axis), axis)

    def any_dn(self, m, axis):
        """m[i] or m[i-1] along the axis for a boolean mask (just m[0] at the
        lower end of a wall-bounded axis)."""
        if axis == AX_Z and self.wall_z:
            out = m.clone()
            out[1:] = m[1:] | m[:-1]
            return out
        return m | _shift(m, -1, axis)

    def d2abs(self, f, axis):
        """Absolute second difference |f[i+1] - 2 f[i] + f[i-1]| along the
        axis; zero on the end planes of a wall-bounded axis, where one of the
        two neighbours does not exist."""
        if axis == AX_Z and self.wall_z:
            d = torch.zeros_like(f)
            d[1:-1] = (f[2:] - 2.0 * f[1:-1] + f[:-2]).abs()
            return d
        return (_shift(f, 1, axis) - 2.0 * f + _shift(f, -1, axis)).abs()

    def mean3(self, f, axis):
        """Average over the three adjacent cells (over the available ones at
        the ends of a wall-bounded axis)."""
        if axis == AX_Z and self.wall_z:
            n = f.shape[0]
            planes = []
            for k in range(n):
                cand = [f[j] for j in (k - 1, k, k + 1) if 0 <= j < n]
                s = cand[0]
                for c in cand[1:]:
                    s = s + c
                planes.append(s / len(cand))
            return torch.stack(planes)
        lo, hi = _shift(f, -1, axis), _shift(f, 1, axis)
        return (lo + f + hi) / 3.0
