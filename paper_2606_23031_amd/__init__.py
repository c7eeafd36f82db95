"""MI355X-native compositional multi-octree sparse-voxel renderer.

The HIP library (csrc/, C ABI in include/dv.h) does all rendering work; the
``dv`` module is a ctypes binding and ``autograd`` wraps forward/backward
for PyTorch (device memory and streams only).
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdvox.so")

__all__ = ["LIB_PATH"]
