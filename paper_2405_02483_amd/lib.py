"""ctypes binding of libstaggermhd.so, the C ABI declared in include/mhd.h.

Argument marshalling only: every computation runs in the HIP kernels of the
library.  Field arguments are sequences of 8 contiguous torch tensors on the
GPU (rho, px, py, pz, e, bx, by, bz) of the context's dtype and
``mhd_field_elems`` elements each (any shape).  If the library has not been
built, importing this module raises; there is no CPU fallback.
"""
import ctypes
import os

import torch

__all__ = [
    "MHD_OK", "MHD_EINVAL", "MHD_ENOMEM", "MHD_EHIP", "MHD_EDTYPE",
    "MHD_ENONFINITE", "MHD_EUNSUPPORTED", "MHD_F32", "MHD_F64",
    "MHD_BC_PERIODIC", "MHD_BC_WALL", "T_CONT", "T_ADV", "T_PRES", "T_VISC",
    "T_LORENTZ", "T_INDUCT", "T_RESIST", "T_EDIFF", "T_GRAV", "T_ALL", "T_COOL", "T_CORI",
    "T_EDIFFAV", "T_LNP", "T_DIVB", "T_SMAG", "T_MAX5", "T_QUENCH", "T_ORDER2",
    "MhdBox", "MhdParams", "MhdStats", "MhdError", "lib_path", "load",
    "mhd_init", "mhd_destroy", "mhd_last_error", "mhd_field_elems",
    "mhd_box_offset", "mhd_rhs", "mhd_rhs_noalloc", "mhd_step", "mhd_step_adjoint", "mhd_divb_clean",
    "mhd_reductions", "mhd_profile", "mhd_profile_read", "mhd_last_dt", "mhd_set_tile",
    "mhd_set_launch", "mhd_get_launch", "mhd_set_final_tile", "mhd_get_final_tile",
    "mhd_autotune", "mhd_rhs_adjoint",
    "PASS_NAMES", "TILES", "Context",
]

MHD_OK, MHD_EINVAL, MHD_ENOMEM, MHD_EHIP, MHD_EDTYPE, MHD_ENONFINITE, MHD_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
MHD_F32, MHD_F64 = 0, 1
MHD_BC_PERIODIC, MHD_BC_WALL = 0, 1
T_CONT, T_ADV, T_PRES, T_VISC, T_LORENTZ, T_INDUCT, T_RESIST, T_EDIFF, T_GRAV = \
    (1 << i for i in range(9))
T_ALL = (1 << 9) - 1
T_COOL = 1 << 9      # Newtonian cooling; not part of T_ALL
T_CORI = 1 << 10     # Coriolis force; not part of T_ALL
T_EDIFFAV = 1 << 11  # with T_EDIFF: diffusion about the horizontal mean; not part of T_ALL
T_LNP = 1 << 12      # with T_PRES: grad P through ln(P / P_aver); not part of T_ALL
T_DIVB = 1 << 13     # div B diffusion (needs the step's dt); not part of T_ALL
T_SMAG = 1 << 14     # Smagorinsky viscosity added to the speed-like one; not part of T_ALL
T_MAX5 = 1 << 15     # viscosity spread by the maximum over five cells; not part of T_ALL
T_QUENCH = 1 << 16   # quenching of the viscous stress (eq. quench); not part of T_ALL
T_ORDER2 = 1 << 17   # second-order strain where the state is rough; not part of T_ALL


class MhdBox(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("ngz", ctypes.c_int32), ("bc_z", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("Lx", ctypes.c_double), ("Ly", ctypes.c_double), ("Lz", ctypes.c_double),
                ("zc", ctypes.POINTER(ctypes.c_double))]


class MhdParams(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("nbox", ctypes.c_int32),
                ("boxes", ctypes.POINTER(MhdBox)),
                ("gamma", ctypes.c_double), ("mu", ctypes.c_double), ("gz", ctypes.c_double),
                ("nu1", ctypes.c_double), ("nu2", ctypes.c_double), ("nu3", ctypes.c_double),
                ("nu_const", ctypes.c_double), ("c1", ctypes.c_double), ("nuE", ctypes.c_double),
                ("nuB", ctypes.c_double), ("eta_const", ctypes.c_double),
                ("Cdt", ctypes.c_double), ("Cdtd", ctypes.c_double), ("Cdtr", ctypes.c_double),
                ("terms", ctypes.c_uint32), ("reserved", ctypes.c_int32),
                ("e_cool", ctypes.c_double), ("t_cool", ctypes.c_double),
                ("rho_cool", ctypes.c_double), ("cool_cut", ctypes.c_int32),
                ("reserved2", ctypes.c_int32), ("omega", ctypes.c_double * 3),
                ("c_divb", ctypes.c_double), ("c_smag", ctypes.c_double),
                ("q_max", ctypes.c_double), ("q_lim", ctypes.c_double),
                ("d2_lim", ctypes.c_double)]


class MhdStats(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("mom", ctypes.c_double * 3),
                ("ekin", ctypes.c_double), ("emag", ctypes.c_double), ("eint", ctypes.c_double),
                ("divb_max", ctypes.c_double), ("divb_rms", ctypes.c_double),
                ("bmax", ctypes.c_double), ("umax", ctypes.c_double), ("cmax", ctypes.c_double),
                ("numax", ctypes.c_double), ("ratemax", ctypes.c_double), ("dt", ctypes.c_double),
                ("dt_wave", ctypes.c_double), ("dt_diff", ctypes.c_double),
                ("dt_rate", ctypes.c_double), ("dt_argmax", ctypes.c_int64),
                ("dt_box", ctypes.c_int32), ("dt_limit", ctypes.c_int32),
                ("n_nonfinite", ctypes.c_int64), ("n_nonpositive", ctypes.c_int64)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if name == "mom" else v
        return d


class MhdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("mhd error %d: %s" % (code, msg))
        self.code = code


_HERE = os.path.dirname(os.path.abspath(__file__))


def lib_path():
    """The library to load: $STAGGER_MHD_LIB if set (another build of the same
    ABI), else the in-tree build."""
    return os.environ.get("STAGGER_MHD_LIB") or os.path.join(_HERE, "libstaggermhd.so")


_LIB = None
_P8 = ctypes.c_void_p * 8


def load():
    """Load (once) and return the ctypes handle of the library."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError("libstaggermhd.so is not built (%s); run "
                           "`python -m paper_2405_02483_amd.csrc.build`" % path)
    L = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.mhd_init.argtypes = [ctypes.POINTER(MhdParams), vp, ctypes.POINTER(vp)]
    L.mhd_init.restype = ctypes.c_int
    L.mhd_destroy.argtypes = [vp]
    L.mhd_destroy.restype = None
    L.mhd_last_error.argtypes = [vp]
    L.mhd_last_error.restype = ctypes.c_char_p
    L.mhd_field_elems.argtypes = [vp]
    L.mhd_field_elems.restype = i64
    L.mhd_box_offset.argtypes = [vp, i32]
    L.mhd_box_offset.restype = i64
    L.mhd_rhs.argtypes = [vp, _P8, _P8]
    L.mhd_rhs.restype = ctypes.c_int
    L.mhd_rhs_noalloc.argtypes = [vp, _P8, _P8]
    L.mhd_rhs_noalloc.restype = ctypes.c_int
    L.mhd_step.argtypes = [vp, _P8, _P8, _P8, _P8, ctypes.c_double, i32]
    L.mhd_step.restype = ctypes.c_int
    L.mhd_step_adjoint.argtypes = [vp, _P8, ctypes.c_double, _P8, _P8]
    L.mhd_step_adjoint.restype = ctypes.c_int
    L.mhd_reductions.argtypes = [vp, _P8, ctypes.c_void_p, ctypes.POINTER(MhdStats)]
    L.mhd_reductions.restype = ctypes.c_int
    L.mhd_divb_clean.argtypes = [vp, _P8]
    L.mhd_divb_clean.restype = ctypes.c_int
    L.mhd_last_dt.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.mhd_last_dt.restype = ctypes.c_int
    L.mhd_set_tile.argtypes = [vp, i32]
    L.mhd_set_tile.restype = ctypes.c_int
    L.mhd_rhs_adjoint.argtypes = [vp, _P8, _P8, _P8]
    L.mhd_rhs_adjoint.restype = ctypes.c_int
    L.mhd_set_launch.argtypes = [vp, i32, i32]
    L.mhd_set_launch.restype = ctypes.c_int
    L.mhd_get_launch.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.mhd_get_launch.restype = ctypes.c_int
    L.mhd_set_final_tile.argtypes = [vp, i32]
    L.mhd_set_final_tile.restype = ctypes.c_int
    L.mhd_get_final_tile.argtypes = [vp, ctypes.POINTER(i32)]
    L.mhd_get_final_tile.restype = ctypes.c_int
    L.mhd_autotune.argtypes = [vp, _P8, _P8, i32, ctypes.POINTER(ctypes.c_double)]
    L.mhd_autotune.restype = ctypes.c_int
    L.mhd_profile.argtypes = [vp, i32]
    L.mhd_profile.restype = ctypes.c_int
    L.mhd_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64), i32]
    L.mhd_profile_read.restype = ctypes.c_int
    _LIB = L
    return L


def _check(rc, ctx):
    if rc != MHD_OK:
        msg = load().mhd_last_error(ctx).decode(errors="replace")
        raise MhdError(rc, msg)


# ---------------------------------------------------------------------------
# Thin wrappers with the C names.
def mhd_init(params, stream=None):
    """params: MhdParams (with .boxes set).  Returns the context handle."""
    L = load()
    ctx = ctypes.c_void_p()
    s = ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream().cuda_stream)
    rc = L.mhd_init(ctypes.byref(params), s, ctypes.byref(ctx))
    _check(rc, None)
    return ctx


def mhd_destroy(ctx):
    load().mhd_destroy(ctx)


def mhd_last_error(ctx):
    return load().mhd_last_error(ctx).decode(errors="replace")


def mhd_field_elems(ctx):
    return int(load().mhd_field_elems(ctx))


def mhd_box_offset(ctx, b):
    return int(load().mhd_box_offset(ctx, b))


def _ptrs(ts, n, dtype, name):
    if ts is None:
        return None
    if len(ts) != 8:
        raise ValueError("%s: need 8 arrays" % name)
    for t in ts:
        if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and t.numel() == n):
            raise ValueError("%s: need contiguous %s GPU tensors of %d elements" % (name, dtype, n))
    return _P8(*[t.data_ptr() for t in ts])


def mhd_rhs(ctx, f, dfdt, *, dtype, n):
    _check(load().mhd_rhs(ctx, _ptrs(f, n, dtype, "f"), _ptrs(dfdt, n, dtype, "dfdt")), ctx)


def mhd_rhs_noalloc(ctx, f, dfdt, *, dtype, n):
    _check(load().mhd_rhs_noalloc(ctx, _ptrs(f, n, dtype, "f"), _ptrs(dfdt, n, dtype, "dfdt")), ctx)


def mhd_divb_clean(ctx, f, *, dtype, n):
    _check(load().mhd_divb_clean(ctx, _ptrs(f, n, dtype, "f")), ctx)


def mhd_step(ctx, f, tmp1, tmp2, du, dt, nsteps, *, dtype, n):
    _check(load().mhd_step(ctx, _ptrs(f, n, dtype, "f"), _ptrs(tmp1, n, dtype, "tmp1"),
                           _ptrs(tmp2, n, dtype, "tmp2"), _ptrs(du, n, dtype, "dU"),
                           float(dt), int(nsteps)), ctx)


def mhd_step_adjoint(ctx, f_n, dt, gbar_in, gbar_out, *, dtype, n):
    _check(load().mhd_step_adjoint(ctx, _ptrs(f_n, n, dtype, "f_n"), float(dt),
                                   _ptrs(gbar_in, n, dtype, "gbar_in"),
                                   _ptrs(gbar_out, n, dtype, "gbar_out")), ctx)


def mhd_reductions(ctx, f, dfdt=None, *, dtype, n, allow_nonfinite=False):
    st = MhdStats()
    pd = _ptrs(dfdt, n, dtype, "dfdt")
    rc = load().mhd_reductions(ctx, _ptrs(f, n, dtype, "f"),
                               ctypes.cast(pd, ctypes.c_void_p) if pd is not None else None,
                               ctypes.byref(st))
    if rc == MHD_ENONFINITE and allow_nonfinite:
        return st.as_dict()
    _check(rc, ctx)
    return st.as_dict()


PASS_NAMES = ("A1", "unused1", "unused2", "A2", "Q", "P", "F", "ghost", "reduce",
              "adjoint")
TILES = {"64x4": 0, "32x8": 1, "16x16": 2, "16x8": 3, "64x8": 4, "32x16": 5}


def mhd_last_dt(ctx):
    v = ctypes.c_double()
    _check(load().mhd_last_dt(ctx, ctypes.byref(v)), ctx)
    return v.value


def mhd_set_tile(ctx, tile):
    _check(load().mhd_set_tile(ctx, int(tile)), ctx)


def mhd_rhs_adjoint(ctx, f, wbar, fbar, *, dtype, n):
    _check(load().mhd_rhs_adjoint(ctx, _ptrs(f, n, dtype, "f"), _ptrs(wbar, n, dtype, "wbar"),
                                  _ptrs(fbar, n, dtype, "fbar")), ctx)


def mhd_set_launch(ctx, tile, persistent):
    _check(load().mhd_set_launch(ctx, int(tile), int(persistent)), ctx)


def mhd_get_launch(ctx):
    t, m = ctypes.c_int32(), ctypes.c_int32()
    _check(load().mhd_get_launch(ctx, ctypes.byref(t), ctypes.byref(m)), ctx)
    return t.value, m.value


def mhd_set_final_tile(ctx, tile):
    _check(load().mhd_set_final_tile(ctx, int(tile)), ctx)


def mhd_get_final_tile(ctx):
    t = ctypes.c_int32()
    _check(load().mhd_get_final_tile(ctx, ctypes.byref(t)), ctx)
    return t.value


def mhd_autotune(ctx, f, dfdt, reps, *, dtype, n):
    ms = (ctypes.c_double * (2 * len(TILES)))()
    _check(load().mhd_autotune(ctx, _ptrs(f, n, dtype, "f"), _ptrs(dfdt, n, dtype, "dfdt"),
                               int(reps), ms), ctx)
    return list(ms)


def mhd_profile(ctx, enable):
    _check(load().mhd_profile(ctx, int(bool(enable))), ctx)


def mhd_profile_read(ctx):
    n = len(PASS_NAMES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(load().mhd_profile_read(ctx, ms, cnt, n), ctx)
    return {name: (ms[q], int(cnt[q])) for q, name in enumerate(PASS_NAMES)}


# ---------------------------------------------------------------------------
_PARAM_KEYS = ("gamma", "mu", "gz", "nu1", "nu2", "nu3", "nu_const", "c1", "nuE", "nuB",
               "eta_const", "Cdt", "Cdtd", "Cdtr")


class Context:
    """Owns one mhd_ctx.  ``boxes``: list of dicts with nx, ny, nz, ngz,
    wall (bool), Lx, Ly, Lz and, for a stretched z, zc (the nz + 2 ngz
    cell-centre heights); ``params``: dict of physical parameters (the
    fields of mhd_params by name, ``terms`` for the term bits, and e_cool,
    t_cool, rho_cool, cool_cut for Newtonian cooling with T_COOL, omega
    (3 values) for the Coriolis force with T_CORI, c_divb for the div B
    diffusion with T_DIVB, c_smag for the Smagorinsky viscosity with
    T_SMAG, q_max and q_lim for the quenching with T_QUENCH, d2_lim for the
    second-order switch with T_ORDER2)."""

    def __init__(self, boxes, params, dtype=torch.float32, terms=T_ALL, stream=None,
                 device="cuda"):
        if isinstance(boxes, dict):
            boxes = [boxes]
        self.dtype = dtype
        self.device = torch.device(device)
        self.boxes = [dict(b) for b in boxes]
        arr = (MhdBox * len(boxes))()
        self._zc_c = []
        for a, b in zip(arr, boxes):
            a.nx, a.ny, a.nz = b["nx"], b["ny"], b["nz"]
            a.ngz = b.get("ngz", 0)
            a.bc_z = MHD_BC_WALL if b.get("wall", False) else MHD_BC_PERIODIC
            a.reserved = 0
            a.Lx, a.Ly, a.Lz = b.get("Lx", 1.0), b.get("Ly", 1.0), b.get("Lz", 1.0)
            zc = b.get("zc")
            if zc is not None:      # stretched z: the cell-centre heights
                zarr = (ctypes.c_double * len(zc))(*[float(v) for v in zc])
                self._zc_c.append(zarr)
                a.zc = ctypes.cast(zarr, ctypes.POINTER(ctypes.c_double))
        self._boxes_c = arr
        p = MhdParams()
        p.dtype = MHD_F32 if dtype == torch.float32 else MHD_F64
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be float32 or float64")
        p.nbox = len(boxes)
        p.boxes = ctypes.cast(arr, ctypes.POINTER(MhdBox))
        defaults = dict(gamma=5.0 / 3.0, mu=1.0, gz=0.0, nu1=0.02, nu2=1.0, nu3=0.02,
                        nu_const=0.0, c1=0.0, nuE=1.0, nuB=1.0, eta_const=0.0,
                        Cdt=0.3, Cdtd=0.7, Cdtr=0.1)
        defaults.update({k: v for k, v in params.items() if k in _PARAM_KEYS})
        for k in _PARAM_KEYS:
            setattr(p, k, float(defaults[k]))
        p.terms = int(params.get("terms", terms))
        p.reserved = 0
        p.e_cool = float(params.get("e_cool", 0.0))
        p.t_cool = float(params.get("t_cool", 1.0))
        p.rho_cool = float(params.get("rho_cool", 1.0))
        p.cool_cut = int(params.get("cool_cut", 0))
        p.reserved2 = 0
        for a, w in enumerate(params.get("omega", (0.0, 0.0, 0.0))):
            p.omega[a] = float(w)
        p.c_divb = float(params.get("c_divb", 0.0))
        p.c_smag = float(params.get("c_smag", 0.0))
        p.q_max = float(params.get("q_max", 8.0))
        p.q_lim = float(params.get("q_lim", 2.0))
        p.d2_lim = float(params.get("d2_lim", 0.3))
        self.params = p
        self.ctx = mhd_init(p, stream)
        self.n = mhd_field_elems(self.ctx)
        self.offsets = [mhd_box_offset(self.ctx, b) for b in range(len(boxes))]

    def close(self):
        if getattr(self, "ctx", None) is not None:
            mhd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- allocation helpers (torch owns all field memory) --------------------
    def empty(self):
        return [torch.empty(self.n, dtype=self.dtype, device=self.device) for _ in range(8)]

    def zeros(self):
        return [torch.zeros(self.n, dtype=self.dtype, device=self.device) for _ in range(8)]

    def upload(self, per_box_fields):
        """per_box_fields: list over boxes of 8 numpy/torch arrays [nzt, ny, nx]."""
        out = self.empty()
        for b, fields in enumerate(per_box_fields):
            o = self.offsets[b]
            for q in range(8):
                src = torch.as_tensor(fields[q]).reshape(-1)
                out[q][o:o + src.numel()].copy_(src.to(self.dtype))
        return out

    def box_view(self, fields, b):
        bx = self.boxes[b]
        nzt = bx["nz"] + 2 * bx.get("ngz", 0)
        o = self.offsets[b]
        n = nzt * bx["ny"] * bx["nx"]
        return [t[o:o + n].view(nzt, bx["ny"], bx["nx"]) for t in fields]

    # -- the entry points ------------------------------------------------------
    def rhs(self, f, dfdt=None):
        dfdt = dfdt if dfdt is not None else self.empty()
        mhd_rhs(self.ctx, f, dfdt, dtype=self.dtype, n=self.n)
        return dfdt

    def rhs_noalloc(self, f, dfdt):
        """mhd_rhs_noalloc: dfdt (caller-allocated) = F(f), with the call's
        scratch in the library's static device array."""
        mhd_rhs_noalloc(self.ctx, f, dfdt, dtype=self.dtype, n=self.n)
        return dfdt

    def divb_clean(self, f):
        """mhd_divb_clean: B of every (periodic) box projected in place onto
        its discretely solenoidal part (eq. clean1, eq. clean2)."""
        mhd_divb_clean(self.ctx, f, dtype=self.dtype, n=self.n)
        return f

    def step(self, f, dt, nsteps=1, work=None):
        work = work or (self.empty(), self.empty(), self.empty())
        mhd_step(self.ctx, f, work[0], work[1], work[2], dt, nsteps, dtype=self.dtype, n=self.n)
        return f

    def step_adjoint(self, f_n, dt, gbar_in, gbar_out=None):
        gbar_out = gbar_out if gbar_out is not None else self.empty()
        mhd_step_adjoint(self.ctx, f_n, dt, gbar_in, gbar_out, dtype=self.dtype, n=self.n)
        return gbar_out

    def rhs_adjoint(self, f, wbar, fbar=None):
        fbar = fbar if fbar is not None else self.empty()
        mhd_rhs_adjoint(self.ctx, f, wbar, fbar, dtype=self.dtype, n=self.n)
        return fbar

    def last_dt(self):
        return mhd_last_dt(self.ctx)

    def set_tile(self, tile):
        mhd_set_tile(self.ctx, TILES[tile] if isinstance(tile, str) else tile)

    def set_launch(self, tile, persistent):
        mhd_set_launch(self.ctx, TILES[tile] if isinstance(tile, str) else tile, persistent)

    def get_launch(self):
        t, m = mhd_get_launch(self.ctx)
        return {v: k for k, v in TILES.items()}[t], m

    def set_final_tile(self, tile):
        """Tile shape of pass F alone (set_tile / set_launch reset it)."""
        mhd_set_final_tile(self.ctx, TILES[tile] if isinstance(tile, str) else tile)

    def get_final_tile(self):
        return {v: k for k, v in TILES.items()}[mhd_get_final_tile(self.ctx)]


    def autotune(self, f, reps=3, dfdt=None):
        """Times RK stages of f in every tile shape and launch mode and keeps
        the fastest (then, possibly, another shape for pass F alone:
        get_final_tile); returns {(tile, persistent): ms per stage} of the
        uniform launches."""
        dfdt = dfdt if dfdt is not None else self.empty()
        ms = mhd_autotune(self.ctx, f, dfdt, reps, dtype=self.dtype, n=self.n)
        names = {v: k for k, v in TILES.items()}
        return {(names[q // 2], q % 2): ms[q] for q in range(2 * len(TILES)) if ms[q] > 0}

    def profile(self, enable=True):
        mhd_profile(self.ctx, enable)

    def profile_read(self):
        return mhd_profile_read(self.ctx)

    def reductions(self, f, dfdt=None, allow_nonfinite=False):
        return mhd_reductions(self.ctx, f, dfdt, dtype=self.dtype, n=self.n,
                              allow_nonfinite=allow_nonfinite)
