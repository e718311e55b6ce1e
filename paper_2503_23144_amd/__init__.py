"""MI355X-native hot path of four-component LR-CCSD polarizabilities.

The compute path is the HIP library ``liblrcc.so`` (C-ABI declared in
``include/lrcc.h``); ``paper_2503_23144_amd.lrcc`` is its thin ctypes
binding.  ``paper_2503_23144_amd.synth`` draws seeded synthetic inputs.
Submodules are imported on demand so that the input generator can be used
on a host without a GPU.
"""
