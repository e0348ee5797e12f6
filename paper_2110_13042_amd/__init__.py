"""MI355X-native AtA: the Gram product C = A^T A of arXiv 2110.13042.

The compute path is the C-ABI library ``libata.so`` (hand-written HIP for
gfx950) declared in ``include/ata.h``; ``ata`` is its thin ctypes binding.
Importing this package does not load the library; the first call does, and
it raises if the library is missing or no GPU is present.
"""
__all__ = ["ata", "workloads"]
