"""Shared helpers of the test suite: conversions between the generators'
numpy arrays, the oracle's float64 CPU tensors and the library's packed GPU
arrays, and the error measure used by every parity test."""
import numpy as np
import torch

import oracle as O


def to_cpu64(f):
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).to(torch.float64) for a in f)


def grid_params(box, prm, **over):
    p = dict(prm)
    p.update(over)
    keys = O.Params.__dataclass_fields__.keys()
    return O.Grid(**box), O.Params(**{k: v for k, v in p.items() if k in keys})


def rel_errors(got, want, floor_frac=1e-3):
    """Per-field relative L2 error ||got - want|| / max(||want||, floor) with
    floor = floor_frac * (largest field norm), so fields that vanish in the
    reference are judged against the scale of the others."""
    gots = [g.detach().to("cpu", torch.float64) for g in got]
    norms = [float(torch.linalg.norm(w)) for w in want]
    big = max(norms) if norms else 0.0
    out = []
    for g, w, n in zip(gots, want, norms):
        d = float(torch.linalg.norm(g.reshape(w.shape) - w))
        out.append(d / max(n, floor_frac * big, 1e-300))
    return out


def interior(f, box):
    g0 = box.get("ngz", 0)
    g1 = g0 + box["nz"]
    return [a[g0:g1] for a in f]
