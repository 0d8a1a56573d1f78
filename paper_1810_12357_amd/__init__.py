"""MI355X (gfx950) electronic-temperature sub-step of the meshless
two-temperature MD scheme (Ullah & Ponga, arXiv 1810.12357).

The computation lives in the C-ABI library libl2t.so (include/l2t.h, HIP
kernels under csrc/); ``l2t`` is its ctypes binding and ``autograd`` wraps the
adjoint entry points in a torch.autograd.Function.
"""
from . import l2t  # noqa: F401  (the shared library itself loads on first use)

__all__ = ["l2t"]
