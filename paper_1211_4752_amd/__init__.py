"""MI355X-native level-dependent complex-shifted multigrid for indefinite Helmholtz.

The compute path is a HIP (gfx950) shared library behind a C ABI declared in
include/mg.h; ``paper_1211_4752_amd.mg`` is the thin ctypes binding that
marshals torch device tensors into it.  Importing the package does not load
the library: ``paper_1211_4752_amd.mg.lib()`` does, and raises if it is
missing.
"""

__all__ = ["mg", "workloads"]
