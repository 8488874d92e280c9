"""MI355X-native differentiable 2D Gaussian surfel rasterizer (the 2DGS
mapping backend's hot path of Flash-Mono, arXiv 2604.03092).

The compute lives in ``libfm2dgs.so`` (HIP, gfx950), built in-tree by
``python -m paper_2604_03092_amd.build``; ``raster`` binds it to PyTorch
tensors and ``scenes`` draws the seeded synthetic workloads.  Importing the
package loads nothing; the library is loaded (and must exist) on first use.
"""
__all__ = ["build", "native", "raster", "scenes"]
