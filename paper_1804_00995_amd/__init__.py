"""MI355X-native H-matrix BEM operators (Helmholtz / Laplace single layer and its gradient
kernels at quadrature points), with the Galerkin P1 system and the RWG EFIE/MFIE/CFIE on top.

The compute path is the HIP library ``libhmx.so`` built from ``csrc/``; ``hmx`` is its thin
ctypes binding.  Importing the package loads nothing; ``from paper_1804_00995_amd import hmx``
loads the library and fails loudly if it is missing.
"""
__all__ = ["inputs", "hmx"]
