"""One checkpointed adjoint of a short rollout, for profiling runs:

    python -m paper_2405_02483_amd.adjoint_probe [--size 128] [--steps 2]

Runs the turbulent box (seed 4) in float32 forward over the given steps with
mhd_step and then backward with mhd_step_adjoint (via MHDRollout), printing
the wall time of each part.  The rocprofv3 counters of this command give the
bytes the adjoint moves per step."""
import argparse
import json
import time

import torch

from . import inputs
from .lib import Context
from .rollout import rollout


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--steps", type=int, default=2)
    a = ap.parse_args()
    f, box, prm = inputs.turbulent(n=a.size, seed=4)
    ctx = Context(box, prm, dtype=torch.float32)
    x0 = ctx.upload([f])
    dt = ctx.reductions(x0)["dt"]
    x = [t.clone().requires_grad_(True) for t in x0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y = rollout(ctx, x, dt, a.steps, ncheck=a.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    torch.autograd.grad(sum((v * v).sum() for v in y), x)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(json.dumps({"size": a.size, "steps": a.steps, "forward_ms": (t1 - t0) * 1e3,
                      "backward_ms": (t2 - t1) * 1e3}))
    ctx.close()


if __name__ == "__main__":
    main()
