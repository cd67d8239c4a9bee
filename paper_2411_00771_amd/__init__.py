"""MI355X-native differentiable 2D-Gaussian surfel tile rasterizer (CityGaussianV2 hot path).

Submodules:
    scenes   seeded synthetic inputs (no rasterizer arithmetic)
    _lib     ctypes binding of libcgv2r.so (include/cgv2r.h)
    raster   device engine, autograd Functions
    server   continuous-batching render server
The HIP library is loaded on first use; a missing build raises, there is no CPU fallback.
"""
__all__ = ["scenes", "raster", "server"]
