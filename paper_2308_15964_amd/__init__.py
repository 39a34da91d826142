"""spx: tile-DAG Cholesky factorisation and solve on one MI355X (gfx950).

The compute path lives in the HIP library libspx.so (csrc/), reached through the C ABI
declared in include/spx.h; spx.py is the ctypes binding.  Importing this package loads
nothing: the binding loads the library on first use and raises if it is missing.
"""
