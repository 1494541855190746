"""Discrete Morse Sandwich persistence diagrams (D0, D1, D2) of scalar fields
on 3D regular grids, computed by hand-written HIP kernels for MI355X (gfx950)
behind the C ABI in include/dms.h.

``paper_2206_13932_amd.dms`` is the ctypes binding; it loads libdms.so when a
Context is created and raises if the library is not built.
"""
