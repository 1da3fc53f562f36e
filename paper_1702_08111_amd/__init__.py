"""MI355X (gfx950) two-level Method of Local Corrections.

The solver lives in the HIP library libmlc.so (C ABI in include/mlc.h); the
module `paper_1702_08111_amd.mlc` is a thin ctypes binding with the same
names.  Importing this package loads nothing; the binding loads the library
on first use and raises if it is missing (there is no fallback path).
"""
