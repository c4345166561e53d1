"""The seeded input generators (CPU): the recipe each workload states -
shapes, layouts, the closed-form profiles and ratios it promises, and
determinism by seed.  The generators hold none of the method's arithmetic,
so these checks use only numpy."""
import numpy as np
import pytest

from paper_2405_02483_amd import inputs


def test_stratified_profile_and_field():
    nx, ny, nz, ngz = 8, 6, 16, 5
    f, box, prm = inputs.stratified(nx, ny, nz, seed=3, ngz=ngz)
    assert all(a.shape == (nz + 2 * ngz, ny, nx) for a in f)
    assert box["wall"] and box["ngz"] == ngz and "zc" not in box
    H, g = 0.25, prm["gz"]
    assert g == pytest.approx(1.0 / H)
    zc = (np.arange(nz + 2 * ngz) - ngz + 0.5) / nz
    np.testing.assert_allclose(f[0][:, 0, 0], np.exp(-zc / H), rtol=1e-15)
    # isothermal: (gamma - 1) e = rho = P
    np.testing.assert_allclose((prm["gamma"] - 1) * f[4], f[0], rtol=1e-14)
    # beta = 2 mu P / B^2 = 100 at mid-height (P = exp(-2))
    assert 2 * np.exp(-0.5 / H) / f[7][0, 0, 0] ** 2 == pytest.approx(100.0)
    assert np.all(f[5] == 0) and np.all(f[6] == 0)
    # velocity noise of 1e-3 on every face
    u = f[1] / f[0]
    assert 0.5e-3 < float(np.std(u)) < 2e-3


def test_stratified_stretched_heights():
    nx, ny, nz, ngz = 6, 6, 32, 5
    a, b = 0.35, -0.2
    f, box, _ = inputs.stratified(nx, ny, nz, seed=3, ngz=ngz, stretch=(a, b))
    zc = np.array(box["zc"])
    assert zc.shape == (nz + 2 * ngz,)
    assert np.all(np.diff(zc) > 0)
    u = (np.arange(nz + 2 * ngz) - ngz + 0.5) / nz
    np.testing.assert_allclose(zc, u + a * u * (1 - u) + b * u * u * (1 - u), rtol=0, atol=1e-15)
    # the atmosphere sits at the stretched heights
    np.testing.assert_allclose(f[0][:, 0, 0], np.exp(-zc / 0.25), rtol=1e-15)
    # the spacing runs from about 1 + a of the mean at the bottom to about
    # 1 - a - b near the top
    d = np.diff(zc[ngz:ngz + nz]) * nz
    assert d[0] == pytest.approx(1 + a, rel=0.05) and d[-1] == pytest.approx(1 - a - b, rel=0.05)
    # the same seed gives the same noise with and without stretching
    f2, _, _ = inputs.stratified(nx, ny, nz, seed=3, ngz=ngz)
    np.testing.assert_allclose(f[1] / f[0], f2[1] / f2[0], rtol=1e-14, atol=0)


def test_turbulent_mach_beta_and_seed():
    n = 16
    f, box, prm = inputs.turbulent(n=n, seed=2, kmax=4.0)
    rho, px, py, pz, e = f[:5]
    cs = 1.0
    u2 = np.mean(px ** 2 + py ** 2 + pz ** 2)         # p = u at mean density 1
    assert np.sqrt(u2) / cs == pytest.approx(0.5, rel=1e-12)
    p0 = 1.0 / prm["gamma"]
    np.testing.assert_allclose((prm["gamma"] - 1) * e, p0, rtol=1e-15)
    b2 = np.mean(f[5] ** 2 + f[6] ** 2 + f[7] ** 2)
    assert 2 * p0 / b2 == pytest.approx(1.0, rel=1e-12)
    assert 0.005 < float(np.std(rho)) < 0.02
    g, _, _ = inputs.turbulent(n=n, seed=2, kmax=4.0)
    for a, c in zip(f, g):
        np.testing.assert_array_equal(a, c)
    h, _, _ = inputs.turbulent(n=n, seed=3, kmax=4.0)
    assert not np.array_equal(f[1], h[1])


def test_orszag_tang_constants():
    f, box, prm = inputs.orszag_tang_3d(n=8, seed=1)
    np.testing.assert_allclose(f[0], 25 / (36 * np.pi), rtol=1e-15)
    np.testing.assert_allclose((prm["gamma"] - 1) * f[4], 5 / (12 * np.pi), rtol=1e-14)


def test_ensemble_sizes():
    sizes = inputs.ensemble_sizes()
    assert len(sizes) == 96
    assert sorted(set(sizes)) == [48, 64, 80, 96]
    assert all(sizes.count(s) == 24 for s in (48, 64, 80, 96))
    assert sizes == inputs.ensemble_sizes()
    assert sizes != sorted(sizes)
