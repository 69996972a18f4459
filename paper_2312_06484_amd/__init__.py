"""MI355X-native AIRPF (augmented island resampling particle filter) hot path.

The filter runs in hand-written HIP kernels for gfx950 behind a C-ABI
library (include/airpf.h); ``paper_2312_06484_amd.airpf`` is its thin ctypes
binding and ``paper_2312_06484_amd.torch_ops`` its autograd wrapper.
``paper_2312_06484_amd.workloads`` only generates seeded synthetic inputs.
Nothing here is imported eagerly, so importing the input generator does not
load the GPU library.
"""
__all__ = ["airpf", "workloads", "torch_ops", "build"]
