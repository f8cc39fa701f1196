"""MI355X-native w-BFBT Stokes hot path (arXiv 1607.03936): HIP library + thin binding.

The numerical work runs in libwbfbt.so (hand-written HIP kernels for gfx950);
`paper_1607_03936_amd.wbfbt` marshals torch tensors and streams into its C-ABI.
Importing this package does not load the library; the first call does, and
fails loudly if it has not been built.
"""
__all__ = ["wbfbt", "build"]
