"""Seeded synthetic initial states for the five workloads.

This module is shared by the tests, the benchmark and both implementations
(the HIP library and the CPU oracle).  It contains none of the method's
arithmetic: no staggered operator, no equation of the right-hand side.  Fields
are sampled analytically (sinusoids, spectral sums evaluated with numpy FFTs)
at the staggered positions of Section 4.1 of the paper: cell centres at
((i+1/2)dx, (j+1/2)dy, (k+1/2)dz); the x-face of cell (i, j, k) at
(i dx, (j+1/2)dy, (k+1/2)dz), and likewise for y and z.

Every generator returns float64 numpy arrays of shape ``[nzt, ny, nx]`` in the
order ``rho, px, py, pz, e, bx, by, bz`` (``e`` = internal energy per volume),
plus a dict describing the box and the suggested physical parameters.

Workloads (parameters follow the paper's namelist typicals where it gives
them; the rest is stated here):

* ``orszag_tang_3d``  - cyclic 3-D extension of the Orszag-Tang initial state
  (eq. initOT): rho = 25/(36 pi), P = 5/(12 pi), gamma = 5/3, sinusoidal u and B
  of amplitude 1 with seeded phases; each component is independent of its own
  coordinate, so div u = div B = 0 exactly, also discretely.
* ``turbulent``       - random-phase solenoidal u and B with integer wave
  vectors 1 <= |k| <= 8, shell amplitude |k|^-2 for u (rms Mach 0.5 at
  c_s = 1) and |k|^-3 for the vector potential of B (plasma beta 1);
  rho = 1 + 0.01 N(0,1) per cell with uniform internal energy; p = u (mean
  density 1).
* ``stratified``      - isothermal hydrostatic atmosphere along z with 4 scale
  heights (H = Lz/4, g = 1/H, P = rho), 1e-3 N(0,1) velocity noise on every
  face, uniform vertical field with beta = 100 at mid-height, closed walls in
  z with 5 ghost planes per side.
* ``ensemble``        - the turbulent state on a list of uneven cubes.
"""
import numpy as np

__all__ = ["orszag_tang_3d", "turbulent", "stratified", "ensemble_sizes",
           "ensemble", "FIELDS"]

FIELDS = ("rho", "px", "py", "pz", "e", "bx", "by", "bz")


def _coords(n, L, face):
    h = L / n
    i = np.arange(n, dtype=np.float64)
    return (i if face else i + 0.5) * h


def _box(nx, ny, nz, ngz=0, wall=False, L=(1.0, 1.0, 1.0)):
    return dict(nx=nx, ny=ny, nz=nz, ngz=ngz, wall=wall,
                Lx=L[0], Ly=L[1], Lz=L[2])


def orszag_tang_3d(n=32, seed=1, gamma=5.0 / 3.0, amp_u=1.0, amp_b=1.0):
    """3-D Orszag-Tang-like state on an n^3 periodic unit cube."""
    rng = np.random.default_rng(seed)
    phx, phy, phz = rng.random(3)
    twopi = 2.0 * np.pi
    rho0 = 25.0 / (36.0 * np.pi)
    p0 = 5.0 / (12.0 * np.pi)
    xc, xf = _coords(n, 1.0, False), _coords(n, 1.0, True)
    shape = (n, n, n)
    Z, Y, X = 0, 1, 2

    def bc(v, ax):                       # broadcast a 1-D profile along ax
        s = [1, 1, 1]
        s[ax] = n
        return np.broadcast_to(v.reshape(s), shape).copy()

    rho = np.full(shape, rho0)
    e = np.full(shape, p0 / (gamma - 1.0))
    # u_x(y), u_y(z), u_z(x): sampled at the cell-centre coordinate of the
    # axis they depend on (faces only move the component's own coordinate).
    ux = -amp_u * np.sin(twopi * (xc + phy))
    uy = amp_u * np.sin(twopi * (xc + phz))
    uz = amp_u * np.sin(twopi * (xc + phx))
    px = rho0 * bc(ux, Y)
    py = rho0 * bc(uy, Z)
    pz = rho0 * bc(uz, X)
    bx = bc(-amp_b * np.sin(twopi * (xc + phy)), Y)
    by = bc(amp_b * np.sin(2.0 * twopi * (xc + phz)), Z)
    bz = bc(-amp_b * np.sin(twopi * (xc + phx)), X)
    box = _box(n, n, n)
    params = dict(gamma=gamma, mu=1.0, gz=0.0, nu1=0.02, nu2=1.0, nu3=0.02,
                  nuE=1.0, nuB=1.0, c1=0.0, Cdt=0.3, Cdtd=0.7, Cdtr=0.1)
    return [rho, px, py, pz, e, bx, by, bz], box, params


def _kgrid(n):
    k = np.fft.fftfreq(n, d=1.0 / n)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    return KX, KY, KZ


def _random_spectrum(rng, n, kmax, slope):
    """Complex vector spectrum (3, n, n, n), |k| in [1, kmax], amplitude
    |k|^slope, random phases, components Gaussian."""
    KX, KY, KZ = _kgrid(n)
    kk = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    band = (kk >= 1.0) & (kk <= kmax)
    amp = np.zeros_like(kk)
    amp[band] = kk[band] ** slope
    spec = (rng.standard_normal((3,) + kk.shape)
            + 1j * rng.standard_normal((3,) + kk.shape)) * amp
    return spec, (KX, KY, KZ), kk


def _project_solenoidal(spec, K, kk):
    KX, KY, KZ = K
    k2 = np.where(kk > 0, kk ** 2, 1.0)
    kd = (KX * spec[0] + KY * spec[1] + KZ * spec[2]) / k2
    return np.stack([spec[0] - KX * kd, spec[1] - KY * kd, spec[2] - KZ * kd])


def _sample(spec_c, K, n, shift):
    """Real field sum_k c_k exp(2 pi i k.(x + s)) at the centre grid, with the
    sample points moved by ``shift`` (cells, per axis x, y, z)."""
    KX, KY, KZ = K
    ph = np.exp(2j * np.pi * (KX * shift[0] + KY * shift[1] + KZ * shift[2]) / n)
    return np.real(np.fft.ifftn(spec_c * ph)) * n ** 3


# component a lives on the face normal to a: shifted by -1/2 along a
_FACE_SHIFT = {0: (-0.5, 0.0, 0.0), 1: (0.0, -0.5, 0.0), 2: (0.0, 0.0, -0.5)}


def turbulent(n=256, seed=2, gamma=5.0 / 3.0, mach=0.5, beta=1.0, kmax=8.0,
              rho_noise=0.01):
    """Random-phase solenoidal turbulence on an n^3 periodic unit cube."""
    rng = np.random.default_rng(seed)
    rho0, cs = 1.0, 1.0
    p0 = rho0 * cs ** 2 / gamma
    # velocity: |k|^-2 shell amplitude, projected to div u = 0
    su, K, kk = _random_spectrum(rng, n, kmax, -2.0)
    su = _project_solenoidal(su, K, kk)
    u = [_sample(su[a], K, n, _FACE_SHIFT[a]) for a in range(3)]
    urms = np.sqrt(np.mean(u[0] ** 2 + u[1] ** 2 + u[2] ** 2))
    u = [c * (mach * cs / urms) for c in u]
    # field: B = curl A (continuous curl, in Fourier space), |k|^-3 for A
    sa, K, kk = _random_spectrum(rng, n, kmax, -3.0)
    KX, KY, KZ = K
    tw = 2j * np.pi
    sb = np.stack([tw * (KY * sa[2] - KZ * sa[1]),
                   tw * (KZ * sa[0] - KX * sa[2]),
                   tw * (KX * sa[1] - KY * sa[0])])
    b = [_sample(sb[a], K, n, _FACE_SHIFT[a]) for a in range(3)]
    b2 = np.mean(b[0] ** 2 + b[1] ** 2 + b[2] ** 2)
    b = [c * np.sqrt(2.0 * p0 / (beta * b2)) for c in b]
    rho = rho0 + rho_noise * rng.standard_normal((n, n, n))
    e = np.full((n, n, n), p0 / (gamma - 1.0))
    px, py, pz = (rho0 * c for c in u)
    box = _box(n, n, n)
    params = dict(gamma=gamma, mu=1.0, gz=0.0, nu1=0.02, nu2=1.0, nu3=0.02,
                  nuE=1.0, nuB=1.0, c1=0.0, Cdt=0.3, Cdtd=0.7, Cdtr=0.1)
    return [rho, px, py, pz, e, b[0], b[1], b[2]], box, params


def stratified(nx=512, ny=512, nz=512, seed=3, gamma=5.0 / 3.0, ngz=5,
               scale_heights=4.0, noise=1e-3, beta_mid=100.0, stretch=None):
    """Isothermal stratified box with closed z walls (unit cube interior).
    stretch = (a, b): a stretched z axis with heights z = L s(u) at
    u = (k - ngz + 1/2) / nz for the cell centres (k - ngz at the lower
    faces), s(u) = u + a u (1 - u) + b u^2 (1 - u), ghost planes included;
    the box then carries the centre heights as zc."""
    rng = np.random.default_rng(seed)
    L = 1.0
    H = L / scale_heights
    g = 1.0 / H                  # P = rho (isothermal, (gamma-1) e_m = 1)
    dz = L / nz
    nzt = nz + 2 * ngz
    kz = np.arange(nzt, dtype=np.float64) - ngz
    if stretch is None:
        zc = (kz + 0.5) * dz     # centre heights, z = 0 at the lower wall
        zf = kz * dz             # lower z-face heights
    else:
        a, b = stretch
        s = lambda u: u + a * u * (1.0 - u) + b * u * u * (1.0 - u)
        zc = L * s((kz + 0.5) / nz)
        zf = L * s(kz / nz)
    rc = np.exp(-zc / H)
    rf = np.exp(-zf / H)
    shape = (nzt, ny, nx)
    rho = np.broadcast_to(rc[:, None, None], shape).copy()
    e = rho / (gamma - 1.0)
    ux = noise * rng.standard_normal(shape)
    uy = noise * rng.standard_normal(shape)
    uz = noise * rng.standard_normal(shape)
    px = rho * ux
    py = rho * uy
    pz = rf[:, None, None] * uz
    pmid = np.exp(-0.5 * L / H)
    bz = np.full(shape, np.sqrt(2.0 * pmid / beta_mid))
    bx = np.zeros(shape)
    by = np.zeros(shape)
    box = _box(nx, ny, nz, ngz=ngz, wall=True, L=(nx * dz, ny * dz, L))
    if stretch is not None:
        box["zc"] = tuple(float(z) for z in zc)
    params = dict(gamma=gamma, mu=1.0, gz=g, nu1=0.02, nu2=1.0, nu3=0.02,
                  nuE=1.0, nuB=1.0, c1=0.0, Cdt=0.3, Cdtd=0.7, Cdtr=0.1)
    return [rho, px, py, pz, e, bx, by, bz], box, params


def ensemble_sizes(nbox=96, sizes=(48, 64, 80, 96), seed=5):
    """Box edge lengths: nbox/len(sizes) of each size, order shuffled."""
    per = nbox // len(sizes)
    lst = [s for s in sizes for _ in range(per)]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(lst))
    return [lst[i] for i in perm]


def ensemble(nbox=96, sizes=(48, 64, 80, 96), seed=5):
    """List of (fields, box) for the batched ensemble; box b uses the
    turbulent generator with seed 5000 + b."""
    out = []
    for b, n in enumerate(ensemble_sizes(nbox, sizes, seed)):
        f, box, params = turbulent(n=n, seed=5000 + b)
        out.append((f, box))
    return out, params
