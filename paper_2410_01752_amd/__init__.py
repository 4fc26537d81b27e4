"""SISSO hot path on MI355X (gfx950): feature expansion, SIS screening and the
l0 sparsifying operator as hand-written HIP kernels behind a C ABI
(include/sisso.h).  Importing the package does not load the GPU library;
`paper_2410_01752_amd.fit.Engine` does, and fails loudly if it is missing.
"""
__all__ = ["inputs"]
