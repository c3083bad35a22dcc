"""MI355X-native many-body (EAM / second-moment tight-binding) MD force path.

The compute path lives in the HIP library `libmd.so` (C ABI declared in
include/md.h).  `paper_1212_6332_amd.md` is its thin ctypes binding; it loads
the library lazily so that the input generators in `workloads` can be used
without a GPU.
"""
__all__ = ["workloads"]
