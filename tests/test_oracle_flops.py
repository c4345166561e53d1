"""Instrumented operation count of the right-hand side: the oracle's RHS
run under a torch dispatch mode that counts the elements each arithmetic
ATen operation produces (one per element for add, sub, mul, div, neg,
maximum/minimum, comparisons and selects; sqrt, exp and log counted apart),
per interior cell.  It replaces the flop estimate of the roofline
discussion with a measured count of what the method computes."""
import math

import pytest
import torch
from torch.utils._python_dispatch import TorchDispatchMode

import oracle as O
from paper_2405_02483_amd import inputs

ARITH = {"add", "sub", "mul", "div", "neg", "rsub", "maximum", "minimum", "clamp_min",
         "clamp", "where", "gt", "ge", "lt", "le", "eq", "abs", "relu", "reciprocal", "pow"}
TRANSC = {"sqrt", "exp", "log", "rsqrt"}


class _Count(TorchDispatchMode):
    def __init__(self):
        super().__init__()
        self.arith = 0
        self.transc = 0

    def __torch_dispatch__(self, func, types, args=(), kwargs=None):
        out = func(*args, **(kwargs or {}))
        name = func.__name__.split(".")[0].rstrip("_")
        n = sum(t.numel() for t in (out if isinstance(out, (tuple, list)) else (out,))
                if isinstance(t, torch.Tensor))
        if name in ARITH:
            self.arith += n
        elif name in TRANSC:
            self.transc += n
        return out


def rhs_ops_per_cell(n=16):
    f, box, prm = inputs.turbulent(n=n, seed=2)
    ft = tuple(torch.from_numpy(a) for a in f)
    g = O.Grid(**box)
    p = O.Params(**{k: v for k, v in prm.items() if k in O.Params.__dataclass_fields__})
    with _Count() as c:
        O.rhs(ft, g, p)
    return c.arith / n ** 3, c.transc / n ** 3


def test_rhs_operation_count_per_cell():
    arith, transc = rhs_ops_per_cell()
    print("RHS per cell: %.0f arithmetic element operations, %.0f sqrt/exp/log" % (arith, transc))
    # the staggered stencils alone (about 130 six-point operators, 11 operations
    # each in pair form) set the scale
    assert 1000 < arith < 5000
    assert 5 < transc < 60
