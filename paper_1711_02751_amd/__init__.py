"""MI355X-native IMEX HDG-DG shallow-water step (arXiv:1711.02751).

The compute path is the HIP library libimexhdg.so (built by
``python -m paper_1711_02751_amd.build``); ``imexhdg`` is a thin ctypes
binding to its C ABI (include/imexhdg.h) that uses PyTorch only for device
memory and streams.  ``workloads`` holds the seeded synthetic inputs.
"""
