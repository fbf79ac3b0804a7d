"""MI355X-native differentiable ray marcher for mixtures of volumetric primitives.

The HIP library (``libmvp.so``) is loaded lazily by ``paper_2103_01954_amd._lib``;
importing this package does not touch the GPU.
"""
__all__ = ["scenes"]
