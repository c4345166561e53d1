"""Plain float64 CPU oracle for the staggered-mesh MHD right-hand side and its
low-storage third-order Runge-Kutta advance (Stein, Nordlund, Collet &
Trampedach, "The Stagger Code for Accurate and Efficient, Radiation-Coupled
MHD Simulations", arXiv:2405.02483).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the HIP library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product path (``paper_2405_02483_amd``) never imports, links
or calls anything in here, and this package imports nothing from the product.

Every array operation is a whole-array PyTorch CPU operation in float64
(``torch.roll`` for periodic neighbours, explicit per-plane formulas at the
ends of a wall-bounded z axis).  No blocking, fusion or reordering beyond the
definitions cited in each function.  Reverse-mode derivatives (the discrete
adjoint of one RK step) come from ``torch.autograd`` applied to this same
forward code.

Modules
-------
stagger   1-D staggered derivative / interpolation operators, max3 / mean3
mhd       parameters, grid, right-hand side, ghost-zone fill, RK3 step,
          Courant time step, conserved totals and diagnostics, adjoint
"""
from .stagger import *  # noqa: F401,F403
from .mhd import *  # noqa: F401,F403
