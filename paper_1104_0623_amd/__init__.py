"""FIND selected inversion (diag G, diag G<, nearest-neighbour G/G< and bond
currents) on AMD MI355X: a HIP/gfx950 library behind a C-ABI, with a thin
ctypes binding in :mod:`paper_1104_0623_amd.find`.

Importing this package loads nothing; ``paper_1104_0623_amd.find`` loads the
shared library.
"""
