"""MI355X-native adaptively conditioned conic solver (LP / SOCP).

The solver is a C-ABI shared library of hand-written HIP kernels for gfx950
(`libacs.so`, declared in include/acs.h).  `paper_2103_00736_amd.acs` is the
thin ctypes binding; `paper_2103_00736_amd.synth` draws seeded problems.
Nothing is loaded at import time: the library is opened on first use and a
missing library is an error, never a fallback.
"""
__all__ = ["acs", "synth"]
