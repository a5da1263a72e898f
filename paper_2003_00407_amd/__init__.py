"""Batched adaptive-local-basis (ALB) generation on AMD MI355X (gfx950).

The compute path is the HIP library ``libdgalb.so`` (C ABI in
``include/dg_alb.h``); ``dgalb`` is its ctypes binding.
"""
__all__ = ["dgalb"]
