"""MI355X-native Cartesian FMM / Barnes-Hut (arXiv 2005.12351).

The compute lives in ``libfmm.so`` (HIP kernels for gfx950 behind a C ABI,
see ``include/fmm.h``); ``paper_2005_12351_amd.fmm`` is the thin Python
binding.  ``paper_2005_12351_amd.workloads`` draws the seeded synthetic
inputs.  Importing the package does not load the GPU library.
"""
