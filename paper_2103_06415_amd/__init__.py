"""Strongly coupled immersed-boundary flow step for MI355X (gfx950).

The compute path is the HIP library ``lib/libibfsi.so`` (sources in ``csrc/``,
C-ABI in ``include/ibfsi.h``); ``binding`` is its ctypes marshalling layer.
"""
