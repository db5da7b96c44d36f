"""MI355X-native SVT linearized track fit (arXiv:1311.0380, Sec. 2).

The compute path is the HIP library `libsvt.so` behind the C ABI declared in
include/svt.h; `paper_1311_0380_amd.svt` is its ctypes binding.  Submodules
are imported lazily so that the input generators can be used without loading
the GPU library.
"""
__all__ = ["svt", "synth"]
