"""MI355X-native layout-aware copy of nested records (LLAMA, arXiv 2106.04284).

The copy itself runs in ``libllama_mi355x.so`` (HIP kernels for gfx950 behind a
C ABI, declared in ``include/llama_mi355x.h``); ``paper_2106_04284_amd.llama``
is the thin ctypes binding.  Importing the package loads nothing: the shared
library is opened on first use and a missing build raises an error.
"""
