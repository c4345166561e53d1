"""Throughput of the staggered-MHD RK3 step on one MI355X.

Workload (default): the 512^3 stratified box - isothermal hydrostatic
atmosphere with 4 scale heights, constant gravity along z, 1e-3 velocity
noise, uniform vertical field (beta = 100 at mid-height), periodic x and y,
closed walls in z with 5 ghost planes per side - in float32, every term of
the right-hand side on.  One timed step is a full RK3 step with its own
Courant time step: mhd_step(dt = 0, 1), which computes the float64 Courant
dt of the step's initial state on the device during the first stage.
Inputs are resident in HBM before timing.

Prints ONE JSON line:  metric, value (interior cell-updates/s per RK step),
ms_per_step, the float64 figures of the same workload, the roofline of the
RK stage (algorithmic bytes per stage / measured stage time, HIP events on
the library's stream; beside the 8 TB/s peak, the bandwidth of a plain 1 GiB
device copy measured in the same run, the HBM bytes the counters measured
and the vector-issue ceiling of the counted VALU instructions), the same
float32 workload with each optional term on (Newtonian cooling, the Coriolis
force, energy diffusion about the horizontal mean, the ln(P/P_aver) pressure
gradient, div B diffusion, the Smagorinsky viscosity with the five-cell
maximum, quenching, the second-order switch, a stretched z axis), div B
cleaning of a 256^3 box, the adjoint legs (the 128^3 turbulent box; a 64^3
walled box with every optional term) and the ensemble leg, and the CPU oracle
timed on a bounded sample: one RK step of a full-height column window of the
same state, whose central columns the float32 step of the whole box is
compared with, field by field.

    python bench.py [--steps K] [--warmup W] [--size N] [--no-fp64]
                    [--no-cpu-baseline] [--no-adjoint] [--no-sources] [--tile TXxTY]
    python bench.py --adjoint-only  (the adjoint leg alone, for profiling)
    python bench.py --clean-only    (the div B cleaning leg alone, for profiling)
    python bench.py --fp64-only     (the float64 step alone, for profiling)
    python bench.py --cpu-table     (the CPU oracle alone, 32^3..256^3)
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
# Vector issue rate: 256 CUs x 4 SIMDs, a wave64 VALU instruction every 4
# cycles per SIMD (16 lanes; no packed math) at 2.4 GHz = 3.93e13
# lane-instructions/s (the 78.6 TFLOP/s of unpacked float32 FMAs).
VALU_LANE_RATE = 256 * 4 * 16 * 2.4e9
# The float32 step's check against the oracle: one full-height window of
# the state, periodic in x and y, WIN_MARGIN columns each side of a central
# WIN_CORE x WIN_CORE block (one RK step reaches at most 3 x 14 cells).
WIN_MARGIN, WIN_CORE = 44, 16
# Algorithmic HBM words per interior cell per RK stage (8 fields, 2N storage,
# stage input and output in different buffers): stage 1 reads f, writes dU
# and f; stage 2 reads f and dU, writes dU and f; stage 3 reads f and dU,
# writes f.  80 words per full step.
WORDS_PER_STAGE = (24, 32, 24)
STAGE_PASSES = ("A1", "A2", "Q", "P", "F")
# Newtonian cooling for the stratified workload: toward the atmosphere's own
# energy per unit mass (1 / (gamma - 1)), with the low-density cut-off at the
# mid-height density exp(-2)
COOLING = dict(e_cool=1.5, t_cool=0.1, rho_cool=math.exp(-2.0), cool_cut=1)
# Coriolis force: a rotation vector of magnitude 1 tilted 30 degrees from z
# toward y (a box at 60 degrees latitude)
CORIOLIS = dict(omega=(0.0, 0.5, math.sqrt(3.0) / 2.0))
# Stretched z axis for the stratified workload: the cubic height map's
# coefficients (a, b); the spacing falls from 1.35 of the mean at the bottom
# to about 0.85 near the top
STRETCH = (0.35, -0.2)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash(root=ROOT):
    """Hash of what builds the forward stage kernels: their sources without
    `//` comments and blank lines, and the build flags (the adjoint's and
    the div B cleaning's own sources are left out).  The committed traffic
    counters are used only while it matches."""
    h = hashlib.sha256()
    d = os.path.join(root, "paper_2405_02483_amd", "csrc")
    for name in sorted(os.listdir(d)):
        if name.startswith(("mhd_adjoint.", "mhd_clean.")):
            continue
        if name.endswith((".hip", ".hpp")) or name == "build.py":
            for line in open(os.path.join(d, name), encoding="utf-8"):
                code = (line.split("#", 1)[0] if name.endswith(".py") else line.split("//", 1)[0]).strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def _profile_record(name):
    """A committed rocprofv3 counter summary (profiles/<name>.json), if it
    was taken from the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except ValueError:
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec


def measured_traffic(dtype_name):
    """HBM bytes per RK stage from the committed counter summary, or None."""
    rec = _profile_record("traffic_rk_stage_stratified512")
    v = (rec or {}).get(dtype_name, {}).get("bytes_per_stage")
    return float(v) if v else None


def measured_valu(dtype_name):
    """VALU lane-instructions per cell and stage from the committed counter
    summary, or None."""
    rec = _profile_record("instructions_rk_stage_stratified512")
    v = (rec or {}).get(dtype_name, {}).get("valu_per_cell_stage")
    return float(v) if v else None


def stage_times(prof, steps):
    """From the library's pass timings over `steps` RK steps ({pass: (total
    ms, intervals)}): ms per RK stage of each pass that ran, with its
    interval count, and the stage time (the sum over STAGE_PASSES).  A pass
    may be timed in more than one interval of a stage (A2 on both sides of
    the Courant dt kernel; Q on both sides of pass P with the second-order
    switch), so the totals are divided by the stages, not the intervals."""
    nst = 3 * steps
    passes = {k: (v[0] / nst, v[1]) for k, v in prof.items() if v[1]}
    stage = sum(prof[p][0] for p in STAGE_PASSES if p in prof) / nst
    return passes, stage


def make_state(workload, size, **kw):
    from paper_2405_02483_amd import inputs
    if workload == "stratified":
        return inputs.stratified(size, size, size, seed=3, **kw)
    if workload == "turbulent":
        return inputs.turbulent(n=size, seed=2)
    raise ValueError(workload)


def _window(f_np, box, x0, y0, width):
    """A full-height column window of the state, periodic in x and y."""
    import numpy as np
    ix = (np.arange(width) + x0) % box["nx"]
    iy = (np.arange(width) + y0) % box["ny"]
    sub = [np.ascontiguousarray(np.asarray(a)[:, iy][:, :, ix]) for a in f_np]
    wbox = dict(box, nx=width, ny=width, Lx=box["Lx"] * width / box["nx"],
                Ly=box["Ly"] * width / box["ny"])
    return sub, wbox


def run_gpu(size, dtype, steps, warmup, workload="stratified", tile=None, over=None,
            launch=None, window=None, state_kw=None, final_tile=None):
    """Times `steps` RK steps.  over: parameters replacing the workload's;
    launch: a (tile, persistent, final-pass tile) to use instead of tuning;
    window: (x0, y0) of a column window: after the timing, one step of the
    initial state with its Courant dt, whose central columns are returned
    (with the window of the initial state and the dt) for the oracle."""
    import numpy as np
    import torch
    from paper_2405_02483_amd.lib import Context

    log("generating the %d^3 %s state" % (size, workload))
    f_np, box, prm = make_state(workload, size, **(state_kw or {}))
    prm = dict(prm, **(over or {}))
    ctx = Context(box, prm, dtype=dtype)
    f = ctx.upload([f_np])
    win = None
    if window is not None:
        win = _window(f_np, box, window[0], window[1], 2 * WIN_MARGIN + WIN_CORE)
        f0 = [t.clone() for t in f]
    del f_np
    tune = None
    if launch is not None:
        ctx.set_launch(launch[0], launch[1])
        ctx.set_final_tile(launch[2])
    elif tile is None:
        tune = ctx.autotune(f, reps=3)          # tile shape and launch mode
    else:
        ctx.set_launch(tile, 0)
        if final_tile is not None:
            ctx.set_final_tile(final_tile)
    work = (ctx.empty(), ctx.empty(), ctx.empty())
    torch.cuda.synchronize()
    ncell = size ** 3

    def one_step():
        ctx.step(f, 0.0, 1, work=work)          # Courant dt on the device

    log("warmup %d steps (%s)" % (warmup, dtype))
    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    ctx.profile(True)
    log("timing %d steps" % steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    gpu_win = None
    if win is not None:
        # one step of the initial state in the launch just timed
        ctx.step(f0, 0.0, 1, work=work)
        nzt = box["nz"] + 2 * box.get("ngz", 0)
        core = np.arange(WIN_MARGIN, WIN_MARGIN + WIN_CORE)
        ix = torch.from_numpy((core + window[0]) % box["nx"]).to(f0[0].device)
        iy = torch.from_numpy((core + window[1]) % box["ny"]).to(f0[0].device)
        gpu_win = dict(sub=win[0], box=win[1], prm=prm, dt=ctx.last_dt(), window=window,
                       got=[t.view(nzt, box["ny"], box["nx"])[:, iy][:, :, ix].double().cpu().numpy()
                            for t in ctx.box_view(f0, 0)])
        del f0
    launch = ctx.get_launch()
    ftile = ctx.get_final_tile()
    dt_last = ctx.last_dt()
    s_end = ctx.reductions(f)
    ctx.close()
    del f, work
    torch.cuda.empty_cache()
    ms = (t1 - t0) * 1e3 / steps
    passes, stage_ms = stage_times(prof, steps)
    return dict(ms_per_step=ms, value=ncell * steps / (t1 - t0), stage_ms=stage_ms,
                launch={"tile": launch[0], "persistent": launch[1], "final_pass_tile": ftile},
                autotune_ms_per_stage=None if tune is None else {
                    "%s/%s" % (k[0], "persistent" if k[1] else "grid"): round(v, 4)
                    for k, v in tune.items()},
                passes=passes,
                dt_last=dt_last, mass=s_end["mass"], ncell=ncell, window=gpu_win)


def stream_copy_gbs(nbytes=1 << 30, reps=10):
    """Achievable HBM bandwidth on this device: a plain device-to-device copy
    of nbytes (read once, written once), timed with HIP events on torch's
    current stream; GB/s counts the bytes read plus the bytes written."""
    import torch
    a = torch.ones(nbytes // 4, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / sec / 1e9


def run_adjoint(n=128, nsteps=40, ncheck=None, dtype_name="f32", stratified=False):
    """Gradient of a linear functional of the state after nsteps RK steps on
    the n^3 turbulent box (seed 4): forward time vs checkpointed backward.
    ncheck None: as many checkpoints as half the free device memory holds.
    stratified: the n^3 stratified box instead (closed walls, 2 x 5 ghost
    planes) with every optional term on (the second-order switch at its
    namelist limit)."""
    import torch
    from paper_2405_02483_amd import inputs
    from paper_2405_02483_amd.lib import (Context, T_ALL, T_COOL, T_CORI, T_EDIFFAV, T_LNP, T_DIVB,
                                          T_SMAG, T_MAX5, T_QUENCH, T_ORDER2)
    from paper_2405_02483_amd.rollout import checkpoint_budget, reversal_cost, rollout
    dtype = torch.float32 if dtype_name == "f32" else torch.float64
    if stratified:
        f, box, prm = inputs.stratified(n, n, n, seed=3)
        prm = dict(prm, **COOLING, **CORIOLIS, terms=T_ALL | T_COOL | T_CORI | T_EDIFFAV | T_LNP | T_DIVB | T_SMAG
                   | T_MAX5 | T_QUENCH | T_ORDER2, c_divb=0.05, c_smag=0.15, q_max=8.0, q_lim=2.0, d2_lim=0.3)
    else:
        f, box, prm = inputs.turbulent(n=n, seed=4)
    ctx = Context(box, prm, dtype=dtype)
    x0 = ctx.upload([f])
    dt = ctx.reductions(x0)["dt"]
    if ncheck is None:
        ncheck = checkpoint_budget(ctx, nsteps)
    w = [torch.ones_like(t) for t in x0]
    x = [t.clone().requires_grad_(True) for t in x0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y = rollout(ctx, x, dt, nsteps, ncheck=ncheck)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss = sum((a * b).sum() for a, b in zip(y, w))
    torch.autograd.grad(loss, x)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ctx.close()
    torch.cuda.empty_cache()
    name = ("stratified_%d (walls, every optional term)" if stratified else "turbulent_%d") % n
    return {"workload": "%s, %d RK steps, %s, %d checkpoints" % (name, nsteps, dtype_name, ncheck),
            "forward_ms": (t1 - t0) * 1e3, "backward_ms": (t2 - t1) * 1e3,
            "adjoint_over_forward": (t2 - t1) / (t1 - t0),
            "recomputed_steps": reversal_cost(nsteps, ncheck)}


def run_ensemble(nbox=96, nsteps=20, ncheck=None):
    """The 96-box ensemble (24 each of 48^3, 64^3, 80^3, 96^3, turbulent
    init, seeds 5000+b), float32, launch autotuned, nsteps steps forward, then
    the checkpointed adjoint of the same rollout."""
    import torch
    from paper_2405_02483_amd import inputs
    from paper_2405_02483_amd.lib import Context
    from paper_2405_02483_amd.rollout import rollout
    log("generating the %d-box ensemble" % nbox)
    cases, prm = inputs.ensemble(nbox=nbox)
    ctx = Context([c[1] for c in cases], prm, dtype=torch.float32)
    x0 = ctx.upload([c[0] for c in cases])
    ncell = sum(c[1]["nx"] * c[1]["ny"] * c[1]["nz"] for c in cases)
    del cases
    tune = ctx.autotune(x0, reps=2)
    dt = ctx.reductions(x0)["dt"]
    work = (ctx.empty(), ctx.empty(), ctx.empty())
    xf = [t.clone() for t in x0]
    ctx.step(xf, dt, 1, work=work)                     # warm-up
    xf = [t.clone() for t in x0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(xf, dt, nsteps, work=work)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    del xf, work
    if ncheck is None:
        from paper_2405_02483_amd.rollout import checkpoint_budget
        ncheck = checkpoint_budget(ctx, nsteps)
    x = [t.clone().requires_grad_(True) for t in x0]
    y = rollout(ctx, x, dt, nsteps, ncheck=ncheck)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    loss = sum((a * a).sum() for a in y)
    torch.autograd.grad(loss, x)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    tile, mode = ctx.get_launch()
    ftile = ctx.get_final_tile()
    ctx.close()
    torch.cuda.empty_cache()
    return {"workload": "%d boxes (48/64/80/96)^3 turbulent, float32, %d RK steps, %d checkpoints"
                        % (nbox, nsteps, ncheck),
            "cells": ncell, "value": ncell * nsteps / (t1 - t0), "unit": "cell-updates/s",
            "forward_ms": (t1 - t0) * 1e3, "rollout_forward_ms": (t2 - t1) * 1e3,
            "backward_ms": (t3 - t2) * 1e3, "adjoint_over_forward": (t3 - t2) / (t1 - t0),
            "launch": {"tile": tile, "persistent": mode, "final_pass_tile": ftile},
            "autotune_ms_per_stage": {"%s/%s" % (k[0], "persistent" if k[1] else "grid"): round(v, 4)
                                    for k, v in tune.items()}}


def run_clean(n=256, reps=5):
    """div B cleaning (mhd_divb_clean) of the n^3 periodic turbulent box in
    float32 with seeded noise added to B: the first call (rocFFT plans,
    scratch) and the mean of `reps` more, and the div B before and after."""
    import numpy as np
    import torch
    from paper_2405_02483_amd import inputs
    from paper_2405_02483_amd.lib import Context
    f, box, prm = inputs.turbulent(n=n, seed=2)
    rng = np.random.default_rng(7)
    for v in (5, 6, 7):
        f[v] = f[v] + 0.01 * rng.standard_normal(f[v].shape).astype(f[v].dtype)
    ctx = Context(box, prm, dtype=torch.float32)
    x = ctx.upload([f])
    del f
    s0 = ctx.reductions(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.divb_clean(x)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s1 = ctx.reductions(x)
    for _ in range(reps):
        ctx.divb_clean(x)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ctx.close()
    torch.cuda.empty_cache()
    h = 1.0 / n
    return {"workload": "turbulent_%d float32 with 1%% noise on B" % n, "first_call_ms": (t1 - t0) * 1e3,
            "ms_per_call": (t2 - t1) * 1e3 / reps,
            "divb_max_dx_over_bmax_before": s0["divb_max"] * h / s0["bmax"],
            "divb_max_dx_over_bmax_after": s1["divb_max"] * h / s1["bmax"]}


def cpu_baseline(win):
    """The float64 CPU oracle on a bounded sample of the same workload: one
    RK step of a full-height column window (periodic in x and y) of the
    benchmark's state, with the dt the library's float32 step took.  The
    window's central columns are exact (they lie beyond the step's reach of
    the window's edges), so they also give the float32 step's error against
    the oracle, field by field (relative L2 over the interior planes)."""
    import numpy as np
    import torch
    import oracle as O
    sub, box, prm, dt = win["sub"], win["box"], win["prm"], win["dt"]
    ft = tuple(torch.from_numpy(np.asarray(a, dtype=np.float64)) for a in sub)
    g = O.Grid(**box)
    p = O.Params(**{k: v for k, v in prm.items() if k in O.Params.__dataclass_fields__})
    t0 = time.perf_counter()
    out = O.step(ft, g, p, dt, 1)
    el = time.perf_counter() - t0
    # the same from the float32-rounded state the library starts from: what
    # the float32 arithmetic adds to the rounding of the stored inputs
    ft32 = tuple(torch.from_numpy(np.asarray(a, dtype=np.float32).astype(np.float64)) for a in sub)
    out32 = O.step(ft32, g, p, dt, 1)
    g0, g1 = box.get("ngz", 0), box.get("ngz", 0) + box["nz"]
    c = slice(WIN_MARGIN, WIN_MARGIN + WIN_CORE)

    def rel(ref):
        errs = {}
        for name, a, b in zip(O.FIELDS, ref, win["got"]):
            want = a[g0:g1, c, c].numpy()
            errs[name] = float(np.linalg.norm(b[g0:g1] - want) / max(np.linalg.norm(want), 1e-300))
        return errs
    errs, errs32 = rel(out), rel(out32)
    ncell = box["nx"] * box["ny"] * box["nz"]
    return {"value": ncell / el, "unit": "cell-updates/s",
            "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": "one RK3 step (float64) of a %dx%d full-height column window (%d interior "
                      "+ 2x%d ghost planes) at (x, y) = %s of the workload's state, %.1f s"
                      % (box["nx"], box["ny"], box["nz"], box.get("ngz", 0), win["window"], el),
            "fp32_vs_oracle": {
                "what": "the library's float32 step of the whole box against the oracle's step "
                        "of the window, on the window's central %dx%d columns, interior planes: "
                        "relative L2 per field (bound 1e-5)" % (WIN_CORE, WIN_CORE),
                "rel_l2": errs, "max": max(errs.values()),
                "rel_l2_from_fp32_rounded_state": errs32,
                "max_from_fp32_rounded_state": max(errs32.values())}}


def cpu_table(sizes=(32, 64, 128, 256)):
    """The float64 CPU oracle's RK-step rate on the stratified workload at
    several sizes, with one thread and with all of torch's threads: the
    median over a few steps (one step at the largest sizes; the single
    thread skips 256^3).  Host-side only."""
    import statistics
    import torch
    import oracle as O
    from paper_2405_02483_amd import inputs
    nthr = torch.get_num_threads()
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    rows = []
    for n in sizes:
        f, box, prm = inputs.stratified(n, n, n, seed=3)
        ft = tuple(torch.from_numpy(a) for a in f)
        g = O.Grid(**box)
        p = O.Params(**{k: v for k, v in prm.items() if k in O.Params.__dataclass_fields__})
        dt = O.courant(ft, g, p)[0]
        for threads in (1, nthr):
            if threads == 1 and n >= 256:
                continue
            torch.set_num_threads(threads)
            steps = 5 if n <= 64 else (3 if n <= 128 else 1)
            if n <= 64:
                O.step(ft, g, p, dt, 1)              # warm-up
            times = []
            for _ in range(steps):
                t0 = time.perf_counter()
                O.step(ft, g, p, dt, 1)
                times.append(time.perf_counter() - t0)
            med = statistics.median(times)
            rows.append({"n": n, "threads": threads, "steps": steps, "median_s_per_step": med,
                         "cell_updates_per_s": n ** 3 / med})
            log("cpu oracle %d^3, %d threads: %.3g s per step" % (n, threads, med))
    torch.set_num_threads(nthr)
    return {"cpu_oracle_table": rows, "host": {"nproc": os.cpu_count(), "torch_threads": nthr,
                                               "cpu": model}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)          # the workload's 50 RK steps
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the adjoint leg, e.g. under a profiler")
    ap.add_argument("--final-tile", default=None,
                    help="with --tile: pass F's own tile shape, e.g. 64x8")
    ap.add_argument("--fp64-only", action="store_true",
                    help="only the float64 step (in the --tile launch if given), e.g. under a profiler")
    ap.add_argument("--clean-only", action="store_true",
                    help="only the div B cleaning leg, e.g. under a profiler")
    ap.add_argument("--adjoint-size", type=int, default=128)
    ap.add_argument("--adjoint-steps", type=int, default=40)
    ap.add_argument("--workload", default="stratified", choices=("stratified", "turbulent"))
    ap.add_argument("--tile", default=None,
                    help="stage kernel tile shape, e.g. 32x8 (default: autotuned)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint and ensemble legs")
    ap.add_argument("--no-sources", action="store_true",
                    help="skip the legs with the optional terms (cooling, Coriolis, energy "
                         "diffusion about the plane mean, ln(P/P_aver) pressure gradient, "
                         "div B diffusion, Smagorinsky with the five-cell maximum, quenching, "
                         "the second-order switch, a stretched z axis) and div B cleaning")
    ap.add_argument("--cpu-table", action="store_true",
                    help="only time the CPU oracle at 32^3..256^3 (1 and all threads); no GPU")
    a = ap.parse_args()
    if a.cpu_table:
        print(json.dumps(cpu_table()), flush=True)
        return
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the hot path would shard by z-slabs or blocks with halo exchange)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.adjoint_only:
        print(json.dumps({"adjoint": run_adjoint(a.adjoint_size, a.adjoint_steps)}), flush=True)
        return
    if a.clean_only:
        print(json.dumps({"divb_clean": run_clean()}), flush=True)
        return
    if a.fp64_only:
        r = run_gpu(a.size, torch.float64, a.steps, a.warmup, a.workload, a.tile, final_tile=a.final_tile)
        print(json.dumps({"fp64": {"ms_per_step": r["ms_per_step"], "value": r["value"],
                                   "stage_ms": r["stage_ms"], "launch": r["launch"]}}), flush=True)
        return

    window = None
    if not a.no_cpu_baseline and a.workload == "stratified" and a.size >= 2 * WIN_MARGIN + WIN_CORE:
        window = (137 % a.size, 301 % a.size)
    r32 = run_gpu(a.size, torch.float32, a.steps, a.warmup, a.workload, a.tile, window=window)
    log("f32: %.2f ms/step, %.3e cell-updates/s" % (r32["ms_per_step"], r32["value"]))
    rsrc = {}
    if not a.no_sources and a.workload == "stratified":
        # the same workload and launch with one more source term switched on
        from paper_2405_02483_amd.lib import (T_ALL, T_COOL, T_CORI, T_EDIFFAV, T_LNP, T_DIVB,
                                              T_SMAG, T_MAX5, T_QUENCH, T_ORDER2)
        L = r32["launch"]
        for name, bit, over, skw in (("cooling", T_COOL, COOLING, None), ("coriolis", T_CORI, CORIOLIS, None),
                                     ("ediffav", T_EDIFFAV, {}, None), ("lnp", T_LNP, {}, None),
                                     ("divb", T_DIVB, dict(c_divb=0.05), None),
                                     ("smagorinsky_max5", T_SMAG | T_MAX5, dict(c_smag=0.15), None),
                                     ("quench", T_QUENCH, dict(q_max=8.0, q_lim=2.0), None),
                                     ("order2", T_ORDER2, dict(d2_lim=0.3), None),
                                     ("stretched", 0, {}, dict(stretch=STRETCH))):
            rsrc[name] = run_gpu(a.size, torch.float32, max(2, a.steps // 5), 1, a.workload,
                                 over=dict(over, terms=T_ALL | bit),
                                 launch=(L["tile"], L["persistent"], L["final_pass_tile"]),
                                 state_kw=skw)
            log("f32 with %s: %.2f ms/step" % (name, rsrc[name]["ms_per_step"]))
    r64 = None
    if not a.no_fp64:
        r64 = run_gpu(a.size, torch.float64, max(2, a.steps // 2), 1, a.workload)
        log("f64: %.2f ms/step, %.3e cell-updates/s" % (r64["ms_per_step"], r64["value"]))

    ncell = r32["ncell"]
    stage_bytes = sum(WORDS_PER_STAGE) / 3.0 * 4 * ncell
    achieved = stage_bytes / (r32["stage_ms"] * 1e-3) / 1e9
    copy_gbs = stream_copy_gbs()
    log("device copy: %.0f GB/s" % copy_gbs)
    traffic = measured_traffic("f32")
    valu = measured_valu("f32")
    out = {
        "metric": "MHD cell-updates/s per RK step at 512^3 FP32 vs FP64; HBM roofline fraction",
        "value": r32["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s_%d" % (a.workload, a.size), "nx": a.size, "ny": a.size,
                   "nz": a.size, "ngz": 5 if a.workload == "stratified" else 0,
                   "boundaries": ("periodic x,y; closed walls z" if a.workload == "stratified"
                                  else "periodic"),
                   "terms": "all", "dt": "Courant (float64, on device) every step"},
        "roofline": {"bound": "hbm", "kernel": "rk_stage (passes: %s)" % "+".join(STAGE_PASSES),
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "algorithmic_bytes_per_stage": stage_bytes,
                     "stage_ms": r32["stage_ms"],
                     "stream_copy_GBs": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs,
                     "traffic_GBs": (None if traffic is None else
                                     traffic / (r32["stage_ms"] * 1e-3) / 1e9),
                     "passes_ms": {k: round(v[0], 4) for k, v in r32["passes"].items()},
                     # the vector-issue ceiling of the same stage: counted VALU
                     # lane-instructions over the chip's issue rate
                     "valu": None if valu is None else {
                         "per_cell_stage": valu,
                         "issue_ms_per_stage": valu * ncell / VALU_LANE_RATE * 1e3,
                         "issue_frac_of_stage": valu * ncell / VALU_LANE_RATE * 1e3 / r32["stage_ms"],
                         "peak_lane_instr_per_s": VALU_LANE_RATE}},
        "launch": r32["launch"],
        "autotune_ms_per_stage": r32["autotune_ms_per_stage"],
    }
    if r64 is not None:
        t64 = measured_traffic("f64")
        out["fp64"] = {"value": r64["value"], "ms_per_step": r64["ms_per_step"],
                       "autotune_ms_per_stage": r64["autotune_ms_per_stage"],
                       # HBM bytes per stage counted in the 16x16 grid launch with
                       # pass F in 64x8 (the autotuner's usual pick for this box)
                       "traffic": t64,
                       "traffic_GBs": None if t64 is None else t64 / (r64["stage_ms"] * 1e-3) / 1e9,
                       "stage_ms": r64["stage_ms"], "launch": r64["launch"],
                       "frac": (2 * stage_bytes / (r64["stage_ms"] * 1e-3) / 1e9) / HBM_PEAK_GBS,
                       "passes_ms": {k: round(v[0], 4) for k, v in r64["passes"].items()}}
        out["fp32_over_fp64"] = r32["value"] / r64["value"]
    what = {
        "cooling": "Newtonian cooling (eq. NewtonCool): e_cool %.1f, t_cool %.1f, low-density "
                   "cut-off at rho_cool = %.4f (mid-height)"
                   % (COOLING["e_cool"], COOLING["t_cool"], COOLING["rho_cool"]),
        "coriolis": "the Coriolis force (eq. mom), Omega = (%.3f, %.3f, %.3f)" % CORIOLIS["omega"],
        "ediffav": "energy diffusion about the horizontal mean (eq. ediffav)",
        "lnp": "the pressure gradient through ln(P/P_aver) (eq. pressure)",
        "divb": "div B diffusion, c_divb 0.05",
        "smagorinsky_max5": "the Smagorinsky viscosity (eq. nusmag, c_smag 0.15) and the maximum "
                            "over five cells (Section 6.1.1)",
        "quench": "quenching of the viscous stress (eq. quench, q_max 8, q_lim 2)",
        "order2": "the second-order switch of the strain (after eq. itv, d2_lim 0.3)",
        "stretched": "a stretched z axis (Section 4.2), heights L s(u), s(u) = u + %.2f u(1-u) %+.2f u^2(1-u): "
                     "dz from %.2f to %.2f of the mean" % (STRETCH[0], STRETCH[1], 1 + STRETCH[0],
                                                           1 - STRETCH[0] - STRETCH[1])}
    for name, r in rsrc.items():
        out[name] = {
            "workload": "%s_%d with %s" % (a.workload, a.size, what[name]),
            "value": r["value"], "unit": "cell-updates/s", "steps": max(2, a.steps // 5),
            "ms_per_step": r["ms_per_step"], "stage_ms": r["stage_ms"],
            "over_plain": r["ms_per_step"] / r32["ms_per_step"],
            "passes_ms": {k: round(v[0], 4) for k, v in r["passes"].items()}}
    if not a.no_sources:
        log("div B cleaning leg")
        out["divb_clean"] = run_clean()
    if not a.no_adjoint:
        log("adjoint leg")
        out["adjoint"] = run_adjoint(a.adjoint_size, a.adjoint_steps)
        log("adjoint leg, walled box with every optional term")
        out["adjoint_walls"] = run_adjoint(64, 20, stratified=True)
        log("ensemble leg")
        out["ensemble"] = run_ensemble()
    if not a.no_cpu_baseline and r32["window"] is not None:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(r32["window"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
