"""MI355X twogrid-preconditioned FGMRES solver for the FE Helmholtz problem.

The solver lives in libhz.so (HIP, gfx950); ``paper_2104_01439_amd.hz`` is its ctypes
binding. Importing this package loads nothing.
"""
