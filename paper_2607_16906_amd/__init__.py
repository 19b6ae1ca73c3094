"""MI355X (gfx950) neural-operator-preconditioned FGMRES for the 2-D Helmholtz equation with PML.

The compute path is the HIP library ``libhzno.so`` (C ABI in ``include/hz.h``);
``paper_2607_16906_amd.hz`` is its thin ctypes binding. Build the library with
``python -m paper_2607_16906_amd.build``.
"""
__all__ = ["hz"]
