"""Local-relaxation message passing for MI355X (gfx950): HIP library + thin binding.

The compute path is liblrh.so (HIP kernels behind a C ABI, include/lrh.h); the module
`paper_2609_40336_amd.lrh` marshals arguments to it.  Nothing here computes on the CPU.
"""
from . import lrh  # noqa: F401

__all__ = ["lrh"]
