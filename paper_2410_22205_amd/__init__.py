"""Narrow-band semi-Lagrangian level-set reconstruction (Preda & Semplice,
arXiv:2410.22205) on AMD Instinct MI355X (gfx950).

The compute path is ``csrc/`` (hand-written HIP behind the C ABI declared in
``include/lsr.h``); :mod:`.lsr` is the thin ctypes binding and :mod:`.synth`
the seeded input generators.  Importing the package loads nothing; the HIP
library is opened on first use of :mod:`.lsr`.
"""
