"""Differentiable multi-step rollout: ``MHDRollout`` wraps ``mhd_step`` and
``mhd_step_adjoint`` in a ``torch.autograd.Function`` with binomial
checkpointing over RK steps (Griewank's recursive reversal schedule).

The forward pass keeps only the initial state.  The backward pass reverses
the steps with at most ``ncheck`` extra stored states, choosing the split
points that minimise the number of recomputed steps (dynamic programme over
(steps, checkpoints)).  All arithmetic runs in the library's kernels: this
module only decides which state to advance from, and when.  The time step is
fixed for the whole rollout and is not differentiated.
"""
import functools

import torch

__all__ = ["MHDRollout", "rollout", "checkpoint_budget", "reversal_cost", "reversal_schedule"]


@functools.lru_cache(maxsize=None)
def _best(n, c):
    """(minimal recomputed steps, first split) to reverse n steps from a
    stored start state with c free checkpoint slots."""
    if n <= 1:
        return 0, 0
    if c == 0:
        return n * (n - 1) // 2, 0
    best = None
    for m in range(1, n):
        cost = m + _best(n - m, c - 1)[0] + _best(m, c)[0]
        if best is None or cost < best[0]:
            best = (cost, m)
    return best


def reversal_cost(nsteps, ncheck):
    """Steps recomputed by the reversal of nsteps steps with ncheck slots."""
    return _best(nsteps, ncheck)[0]


def reversal_schedule(nsteps, ncheck):
    """The sequence of actions of the reversal, as tuples
    ('advance', from_step, to_step) and ('adjoint', step), for inspection
    and tests."""
    acts = []

    def rev(s0, n, c):
        if n == 1:
            acts.append(("adjoint", s0))
            return
        if c == 0:
            for k in range(n - 1, -1, -1):
                if k:
                    acts.append(("advance", s0, s0 + k))
                acts.append(("adjoint", s0 + k))
            return
        m = _best(n, c)[1]
        acts.append(("advance", s0, s0 + m))
        rev(s0 + m, n - m, c - 1)
        rev(s0, m, c)

    if nsteps > 0:
        rev(0, nsteps, ncheck)
    return acts


def _check_dt(dt):
    """The rollout differentiates a fixed step: dt must be a finite positive
    number.  (The library's dt == 0, a Courant step taken on the device,
    changes from step to step and is not differentiated.)"""
    import math
    if not (isinstance(dt, (int, float)) and math.isfinite(dt) and dt > 0):
        raise ValueError("rollout needs a fixed time step dt > 0, got %r" % (dt,))


class _Stepper:
    """Advances copies of states with the library (fixed dt)."""

    def __init__(self, ctx, dt):
        self.ctx = ctx
        self.dt = dt
        self.work = (ctx.empty(), ctx.empty(), ctx.empty())

    def advance(self, x, nsteps):
        y = [t.clone() for t in x]
        if nsteps:
            self.ctx.step(y, self.dt, nsteps, work=self.work)
        return y


class MHDRollout(torch.autograd.Function):
    """y = nsteps RK3 steps of x (8 field tensors of one context)."""

    @staticmethod
    def forward(actx, ctx, dt, nsteps, ncheck, *x):
        _check_dt(dt)
        st = _Stepper(ctx, dt)
        y = st.advance([t.detach() for t in x], nsteps)
        actx.x0 = [t.detach().clone() for t in x]
        actx.lib = ctx
        actx.dt, actx.nsteps, actx.ncheck = dt, nsteps, ncheck
        return tuple(y)

    @staticmethod
    def backward(actx, *gy):
        ctx, dt, nsteps = actx.lib, actx.dt, actx.nsteps
        x0 = actx.x0
        g = [t.contiguous().clone() if t is not None else torch.zeros_like(x0[0]) for t in gy]
        st = _Stepper(ctx, dt)
        tmp = ctx.empty()

        def adjoint(x, g):
            ctx.step_adjoint(x, dt, g, tmp)
            for a, b in zip(g, tmp):
                a.copy_(b)

        def rev(x, n, c):
            if n == 1:
                adjoint(x, g)
                return
            if c == 0:
                for k in range(n - 1, -1, -1):
                    adjoint(st.advance(x, k) if k else x, g)
                return
            m = _best(n, c)[1]
            y = st.advance(x, m)
            rev(y, n - m, c - 1)
            del y
            rev(x, m, c)

        if nsteps > 0:
            rev(x0, nsteps, actx.ncheck)
        return (None, None, None, None) + tuple(g)


def checkpoint_budget(ctx, nsteps, fraction=0.5):
    """Checkpoint slots that fit in `fraction` of the free device memory,
    at most nsteps - 1 (then no step is recomputed)."""
    free, _ = torch.cuda.mem_get_info(ctx.device)
    state = 8 * ctx.n * torch.tensor([], dtype=ctx.dtype).element_size()
    return max(0, min(nsteps - 1, int(fraction * free // state)))


def rollout(ctx, x, dt, nsteps, ncheck=None):
    """Differentiable nsteps-step rollout of the state x (list of 8 tensors).
    ncheck: checkpoint slots for the backward pass; None sizes them from the
    free device memory (checkpoint_budget)."""
    _check_dt(dt)
    if ncheck is None:
        ncheck = checkpoint_budget(ctx, nsteps)
    return list(MHDRollout.apply(ctx, dt, nsteps, ncheck, *x))
