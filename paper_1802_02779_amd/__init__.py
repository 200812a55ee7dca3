"""Store-zechin permanents on MI355X (gfx950).

The compute path is the C-ABI library ``libpermgpu.so`` (hand-written HIP
kernels), declared in ``include/perm.h``.  :mod:`paper_1802_02779_amd.perm`
is its thin Python binding; PyTorch supplies device memory and streams.
"""
__all__ = ["perm", "inputs"]
