"""MI355X-native foveated hybrid renderer (VR-Splatting, Franke, Fink &
Stamminger): a peripheral 3D Gaussian splatting rasterizer, a foveal
neural-point splat into an image pyramid, a small gated-conv decoder and the
foveal/peripheral combination, as hand-written HIP kernels for gfx950 behind
the C-ABI of ``include/vrsplat.h``.

The native library is loaded lazily by :mod:`paper_2410_17932_amd.api`;
importing the package does not touch the GPU.
"""
__all__ = ["synth", "api"]
