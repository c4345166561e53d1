"""Argument checking of mhd_init: every rejected request returns its error
code before any HIP call, so these run without a GPU."""
import ctypes

import pytest

from paper_2405_02483_amd import lib


def _params(**over):
    boxes = over.pop("boxes", [dict(nx=8, ny=8, nz=8, ngz=0, bc_z=0)])
    arr = (lib.MhdBox * len(boxes))()
    keep = [arr]
    for a, b in zip(arr, boxes):
        a.nx, a.ny, a.nz = b["nx"], b["ny"], b["nz"]
        a.ngz, a.bc_z, a.reserved = b.get("ngz", 0), b.get("bc_z", 0), b.get("reserved", 0)
        a.Lx = a.Ly = a.Lz = b.get("L", 1.0)
        if "zc" in b:
            zarr = (ctypes.c_double * len(b["zc"]))(*b["zc"])
            keep.append(zarr)
            a.zc = ctypes.cast(zarr, ctypes.POINTER(ctypes.c_double))
    p = lib.MhdParams()
    p.dtype = over.pop("dtype", lib.MHD_F64)
    p.nbox = over.pop("nbox", len(boxes))
    p.boxes = ctypes.cast(arr, ctypes.POINTER(lib.MhdBox))
    vals = dict(gamma=5 / 3, mu=1.0, gz=0.0, nu1=0.02, nu2=1.0, nu3=0.02, nu_const=0.0,
                c1=0.0, nuE=1.0, nuB=1.0, eta_const=0.0, Cdt=0.3, Cdtd=0.7, Cdtr=0.1)
    vals.update(over)
    for k, v in vals.items():
        if k == "omega":
            for a in range(3):
                p.omega[a] = v[a]
        elif k not in ("terms", "reserved"):
            setattr(p, k, v)
    p.terms = vals.get("terms", lib.T_ALL)
    p.reserved = vals.get("reserved", 0)
    return p, keep


@pytest.mark.parametrize("over,code", [
    (dict(dtype=7), lib.MHD_EDTYPE),
    (dict(gamma=1.0), lib.MHD_EINVAL),
    (dict(mu=0.0), lib.MHD_EINVAL),
    (dict(nu1=-0.1), lib.MHD_EINVAL),
    (dict(Cdt=float("nan")), lib.MHD_EINVAL),
    (dict(terms=1 << 18), lib.MHD_EINVAL),
    (dict(terms=lib.T_ALL | lib.T_SMAG, c_smag=-0.1), lib.MHD_EINVAL),
    (dict(terms=lib.T_ALL | lib.T_SMAG, c_smag=float("nan")), lib.MHD_EINVAL),
    (dict(terms=lib.T_ALL | lib.T_QUENCH, q_max=0.0, q_lim=2.0), lib.MHD_EINVAL),
    (dict(terms=lib.T_ALL | lib.T_QUENCH, q_max=8.0, q_lim=float("inf")), lib.MHD_EINVAL),
    (dict(terms=lib.T_ALL | lib.T_ORDER2, d2_lim=float("nan")), lib.MHD_EINVAL),
    (dict(terms=lib.T_ALL | lib.T_DIVB, c_divb=-0.1), lib.MHD_EINVAL),
    # above the RK3 real-axis limit of the div B diffusion on cubic cells
    (dict(terms=lib.T_ALL | lib.T_DIVB, c_divb=0.1359), lib.MHD_EINVAL),
    (dict(reserved2=1), lib.MHD_EINVAL),
    (dict(terms=lib.T_ALL | lib.T_COOL, t_cool=0.0), lib.MHD_EINVAL),
    (dict(terms=lib.T_ALL | lib.T_COOL, t_cool=1.0, e_cool=float("nan")), lib.MHD_EINVAL),
    (dict(terms=lib.T_ALL | lib.T_COOL, t_cool=1.0, cool_cut=3), lib.MHD_EINVAL),
    (dict(terms=lib.T_ALL | lib.T_COOL, t_cool=1.0, cool_cut=1, rho_cool=0.0), lib.MHD_EINVAL),
    (dict(terms=lib.T_ALL | lib.T_CORI, omega=(0.0, float("inf"), 0.0)), lib.MHD_EINVAL),
    (dict(nbox=0), lib.MHD_EINVAL),
    (dict(boxes=[dict(nx=5, ny=8, nz=8)]), lib.MHD_EINVAL),
    (dict(boxes=[dict(nx=8, ny=8, nz=8, ngz=5, bc_z=0)]), lib.MHD_EINVAL),
    (dict(boxes=[dict(nx=8, ny=8, nz=8, ngz=4, bc_z=1)]), lib.MHD_EINVAL),
    (dict(boxes=[dict(nx=8, ny=8, nz=6, ngz=7, bc_z=1)]), lib.MHD_EINVAL),
    (dict(boxes=[dict(nx=8, ny=8, nz=8, bc_z=3)]), lib.MHD_EINVAL),
    (dict(boxes=[dict(nx=8, ny=8, nz=8, L=0.0)]), lib.MHD_EINVAL),
    # a stretched z axis needs walls and increasing heights
    (dict(boxes=[dict(nx=8, ny=8, nz=8, zc=[0.1 * k for k in range(8)])]), lib.MHD_EINVAL),
    (dict(boxes=[dict(nx=8, ny=8, nz=8, ngz=5, bc_z=1, zc=[0.1 * k * (-1) ** k for k in range(18)])]),
     lib.MHD_EINVAL),
    (dict(boxes=[dict(nx=8, ny=8, nz=8, ngz=5, bc_z=1, zc=[0.1 * k for k in range(17)] + [float("nan")])]),
     lib.MHD_EINVAL),
    (dict(boxes=[dict(nx=1300, ny=1300, nz=1300)]), lib.MHD_EINVAL),   # >= 2^31 cells
])
def test_init_rejects_bad_arguments(over, code):
    L = lib.load()
    p, keep = _params(**over)
    ctx = ctypes.c_void_p()
    rc = L.mhd_init(ctypes.byref(p), None, ctypes.byref(ctx))
    assert rc == code
    assert ctx.value is None
    assert len(L.mhd_last_error(None)) > 0


def test_null_arguments():
    L = lib.load()
    ctx = ctypes.c_void_p()
    assert L.mhd_init(None, None, ctypes.byref(ctx)) == lib.MHD_EINVAL
    p, keep = _params()
    assert L.mhd_init(ctypes.byref(p), None, None) == lib.MHD_EINVAL
    null8 = (ctypes.c_void_p * 8)()
    assert L.mhd_rhs(None, null8, null8) == lib.MHD_EINVAL
    assert L.mhd_field_elems(None) == -1
    assert L.mhd_step(None, null8, null8, null8, null8, 1e-3, 1) == lib.MHD_EINVAL
    assert L.mhd_step_adjoint(None, null8, 1e-3, null8, null8) == lib.MHD_EINVAL
    assert L.mhd_rhs_adjoint(None, null8, null8, null8) == lib.MHD_EINVAL
    assert L.mhd_divb_clean(None, null8) == lib.MHD_EINVAL
    assert L.mhd_set_launch(None, 0, 0) == lib.MHD_EINVAL
    t, m = ctypes.c_int32(), ctypes.c_int32()
    assert L.mhd_get_launch(None, ctypes.byref(t), ctypes.byref(m)) == lib.MHD_EINVAL
    assert L.mhd_set_final_tile(None, 0) == lib.MHD_EINVAL
    assert L.mhd_get_final_tile(None, ctypes.byref(t)) == lib.MHD_EINVAL
    assert L.mhd_autotune(None, null8, null8, 1, None) == lib.MHD_EINVAL
    L.mhd_destroy(None)


def test_divb_limit_accepts_the_stable_range():
    """c_divb just below the RK3 limit of the div B diffusion (0.13582 on
    cubic cells) passes the argument checks: the failure, if any, is not
    MHD_EINVAL (without a GPU the device allocation fails instead)."""
    L = lib.load()
    p, keep = _params(terms=lib.T_ALL | lib.T_DIVB, c_divb=0.1358)
    ctx = ctypes.c_void_p()
    rc = L.mhd_init(ctypes.byref(p), None, ctypes.byref(ctx))
    if rc == lib.MHD_OK:
        L.mhd_destroy(ctx)
    assert rc != lib.MHD_EINVAL, L.mhd_last_error(None)


def test_rollout_refuses_a_courant_dt():
    """The rollout differentiates a fixed step: dt == 0 (the library's
    per-step Courant dt) or dt < 0 raises before any library call."""
    from paper_2405_02483_amd.rollout import rollout
    for dt in (0.0, -1e-3, float("nan")):
        with pytest.raises(ValueError):
            rollout(None, [], dt, 3, ncheck=1)
