"""MI355X-native GPUPEGAS timestep (Kulikov, arXiv:1311.0861).

The compute path is the C-ABI library ``libgpupegas.so`` built from
``csrc/`` (HIP kernels for gfx950); ``gpupegas`` is its thin ctypes binding.
``workloads`` builds seeded synthetic initial states.
"""
