"""MI355X library for the parallel-in-time sparse-grid combination method.

The compute path is the HIP library libctm.so (C ABI in include/ctm.h);
`paper_2509_22156_amd.ctm` is its Python binding. Importing the binding
fails loudly when the library has not been built.
"""
__all__ = ["ctm", "build"]
