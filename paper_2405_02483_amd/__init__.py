"""MI355X-native staggered-mesh MHD right-hand side and low-storage RK3
(Stagger Code method, arXiv:2405.02483) behind a small C ABI.

Submodules are imported lazily so that importing the package never loads the
HIP library by itself:

* ``paper_2405_02483_amd.lib``     - ctypes binding of ``libstaggermhd.so``
                                     (the C ABI in ``include/mhd.h``)
* ``paper_2405_02483_amd.inputs``  - seeded synthetic initial states
* ``paper_2405_02483_amd.rollout`` - autograd wrapper with checkpointing
"""
__version__ = "0.1.0"
