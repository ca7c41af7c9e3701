"""MI355X-native Static and DF-P PageRank (hand-written gfx950 HIP kernels).

Submodules:
  prhip     - ctypes binding of the C-ABI library libprhip.so (the product path)
  graphgen  - seeded synthetic graphs and batch updates (no PageRank arithmetic)
  autograd  - torch.autograd.Function over the weighted forward and adjoint

Nothing is imported eagerly, so the generators work on hosts without a GPU.
"""
__all__ = ["prhip", "graphgen"]
