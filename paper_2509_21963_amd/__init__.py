"""IterativeCUR on MI355X (gfx950): a C-ABI library of hand-written HIP kernels and a
thin Python binding.  See `icur.py` for the binding and `csrc/` for the kernels."""
