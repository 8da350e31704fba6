"""MI355X-native ERP Gaussian rasterizer (OmniGS hot path).

The compute path is the HIP library ``libomnigs.so`` behind the C ABI in
``include/omnigs.h``; ``paper_2404_03202_amd.omnigs`` is its thin ctypes
binding.  Submodules are imported on demand so that the seeded scene
generators can be used without the GPU library.
"""
__all__ = ["omnigs", "scenes", "raster", "serve"]
