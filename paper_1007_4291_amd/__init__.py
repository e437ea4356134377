"""helmsweep: moving-PML sweeping preconditioner for the 2D Helmholtz equation on MI355X (gfx950).

The compute path is the HIP library ``libhelmsweep.so`` behind the C-ABI ``include/helmsweep.h``;
``paper_1007_4291_amd.helmsweep`` is its thin ctypes binding.  Build the library with
``python -m paper_1007_4291_amd.build``.
"""
__all__ = ["helmsweep", "build"]
