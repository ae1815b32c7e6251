"""MI355X-native EPIC direct-imaging correlator with in-loop EPICal calibration.

The compute path is a C-ABI shared library of hand-written HIP kernels for
gfx950 (`include/epic.h`); `paper_1603_02126_amd.lib` is its thin ctypes
binding.  Importing the package does not load the library.
"""
__all__ = ["synth", "lib"]
