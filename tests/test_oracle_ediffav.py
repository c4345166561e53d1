"""Pins of the oracle's energy diffusion about the horizontal mean
(eq. ediffav), independent of its code:

* e_m = a(z) (1 + small in-plane fluctuation with zero plane mean): the
  plane mean is a(z) exactly, so the z flux of the fluctuation form keeps
  only the fluctuation's z dependence.  With a fluctuation that does not
  depend on z, the z flux vanishes and only the x and y fluxes of plain
  energy diffusion remain.
* e_m with plane means exactly 1 on every level: the fluctuation form is
  plain energy diffusion.  (The mean of ln e_m would vary with z here, so
  this also fixes the reading: the log of the mean.)
* e_m constant on each plane: no energy diffusion at all, while plain
  energy diffusion moves energy along the mean gradient.
"""
import math

import pytest
import torch

import oracle as O

N = 12


def _coords():
    i = torch.arange(N, dtype=torch.float64)
    c = (i + 0.5) / N
    z = c.reshape(N, 1, 1).expand(N, N, N)
    x = c.reshape(1, 1, N).expand(N, N, N)
    y = c.reshape(1, N, 1).expand(N, N, N)
    return x, y, z


def _state(em):
    x, y, z = _coords()
    rho = 1.0 + 0.2 * torch.cos(2 * math.pi * y)     # varies in the plane only
    zero = torch.zeros_like(rho)
    return (rho, zero, zero, zero, rho * em, zero, zero, zero)


def _de(f, terms):
    return O.rhs(f, O.Grid(N, N, N), O.Params(terms=terms))[4]


def test_plane_means_of_one_give_plain_diffusion():
    x, y, z = _coords()
    em = 1.0 + 0.3 * torch.sin(2 * math.pi * x) * torch.cos(2 * math.pi * z)
    f = _state(em)
    a = _de(f, O.T_EDIFF | O.T_EDIFFAV)
    b = _de(f, O.T_EDIFF)
    assert float((a - b).abs().max()) < 1e-13 * float(b.abs().max())
    assert float(b.abs().max()) > 1e-3


def test_z_independent_fluctuation_has_no_z_flux():
    x, y, z = _coords()
    az = 1.5 + 0.4 * torch.sin(2 * math.pi * z)
    fl = 1.0 + 0.3 * torch.sin(2 * math.pi * x)
    f = _state(az * fl)
    got = _de(f, O.T_EDIFF | O.T_EDIFFAV)
    full = _de(f, O.T_EDIFF)
    assert float((got - full).abs().max()) > 1e-3 * float(full.abs().max())
    # the difference to plain diffusion is the z divergence of the plain z
    # flux (eq. ediffuse, z component), so the fluctuation form has none
    g = O.Grid(N, N, N)
    Ops = g.ops()
    nt, _ = O.smoothed_viscosity(f, g, O.Params())
    rho, em_ = f[0], f[4] / f[0]
    fz = 1.0 * Ops.zdn(rho) * (g.dz * Ops.zdn(nt)) * Ops.zdn(em_) * Ops.ddzdn(torch.log(em_))
    want = full - Ops.ddzup(fz)
    assert float((got - want).abs().max()) < 1e-12 * float(full.abs().max())


def test_plane_constant_energy_does_not_diffuse():
    x, y, z = _coords()
    em = 1.5 + 0.4 * torch.sin(2 * math.pi * z)
    f = _state(em)
    got = _de(f, O.T_EDIFF | O.T_EDIFFAV)
    plain = _de(f, O.T_EDIFF)
    assert float(plain.abs().max()) > 1e-3
    assert float(got.abs().max()) < 1e-12 * float(plain.abs().max())
