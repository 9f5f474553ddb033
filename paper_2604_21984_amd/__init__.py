"""Soft Anisotropic Diagrams (arxiv 2604.21984) hot path on AMD MI355X (gfx950).

The compute lives in ``libsad.so`` (hand-written HIP kernels behind the C ABI of
``include/sad.h``); ``_lib`` is its argument-marshalling binding.  Importing a
submodule that needs the library raises if it has not been built.
"""
__all__ = ["_lib", "autograd", "encode"]
