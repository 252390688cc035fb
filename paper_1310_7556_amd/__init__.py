"""MI355X-native Hough-transform track finder (vote, peaks, rz refinement).

The compute path is libhough.so (hand-written HIP kernels for gfx950 behind
a C ABI, include/hough.h); `hough` is its ctypes binding.  Submodules are
imported lazily so that building or inspecting the package needs no GPU.
"""
__all__ = ["hough", "build"]
