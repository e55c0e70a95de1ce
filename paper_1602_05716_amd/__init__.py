"""MI355X-native exact-energy sequential Metropolis Monte Carlo for
primitive-model electrolytes (Liang, Xing, Li, arXiv:1602.05716).

The compute path is the C-ABI library ``libmc.so`` (HIP, gfx950) declared in
``include/mc.h``; :mod:`paper_1602_05716_amd.mc` is its thin ctypes binding and
:mod:`paper_1602_05716_amd.inputs` builds seeded synthetic starting states.
Importing this package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
__all__ = ["inputs", "mc"]
