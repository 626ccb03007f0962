"""MI355X-native differentiable tile-based 3D Gaussian Splatting rasterizer.

Submodules (imported lazily so that the input generators can be used
without loading the HIP library):
    _lib        ctypes binding of libgs.so (the C ABI of include/gs.h)
    rasterizer  pipeline, fused Adam and the torch.autograd.Function
    scenes      seeded synthetic scenes, cameras and targets
    build       hipcc build of libgs.so for gfx950
"""
__all__ = ['_lib', 'rasterizer', 'scenes', 'build']
