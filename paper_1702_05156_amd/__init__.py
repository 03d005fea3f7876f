"""MI355X-native Dual-Mode Single Gaussian Model (DSGM) background update.

The hot path of Henderson & Vertescher (arXiv:1702.05156, Sec. 2.2-2.3): the
per-pixel dual Gaussian background model update and the 0/255 foreground mask,
as hand-written HIP kernels for gfx950 behind the C ABI of ``include/dsgm.h``
(``libdsgm.so``).  ``paper_1702_05156_amd.dsgm`` is the ctypes binding.
"""
from . import dsgm  # noqa: F401  (fails loudly if libdsgm.so is missing)
from .dsgm import Params, State, forward  # noqa: F401
