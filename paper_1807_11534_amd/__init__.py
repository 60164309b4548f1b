"""MI355X (gfx950) implementation of the restricted-domain dual method for
two-phase segmentation (Spencer, arXiv 1807.11534).

The compute path is the HIP library ``librdseg.so`` (C ABI in
``include/rdseg.h``); ``rdseg`` and ``autograd`` are thin torch bindings.
Importing the package does not load the library; the first call does, and
raises if the library was not built.
"""
__all__ = ["rdseg", "build"]
