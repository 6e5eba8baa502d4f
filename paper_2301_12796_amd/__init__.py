"""Directional TSDF integration, rendering and point-to-plane ICP on AMD MI355X (gfx950).

The compute path lives in ``libdtsdf.so`` (hand-written HIP kernels behind the C ABI of
``include/dtsdf.h``); ``paper_2301_12796_amd.dtsdf`` is its ctypes binding.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdtsdf.so")
