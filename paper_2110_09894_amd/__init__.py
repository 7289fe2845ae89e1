"""Sliced tensor-network amplitude contraction on AMD MI355X (gfx950).

The compute path lives in the HIP/C++ library ``libqxtn.so`` behind the C-ABI
declared in ``include/qxtn.h``; ``qxtn`` is its ctypes binding.
"""
from . import qxtn  # noqa: F401
from .qxtn import Plan, QxError, permute_c64, cgemm, last_error  # noqa: F401
