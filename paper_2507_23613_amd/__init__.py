"""MI355X-native Multi-Frequency WaveHoltz (MFWH) hot path.

The compute lives in the HIP library ``libmfwh.so`` (C ABI: include/mfwh.h);
``_lib`` is its thin ctypes binding and ``problem.GpuProblem`` sets up one
problem on the GPU.  ``inputs`` draws the seeded synthetic workloads.
Importing this package does not load the library; importing ``_lib`` does
and fails loudly if it has not been built.
"""
__all__ = ["inputs"]
