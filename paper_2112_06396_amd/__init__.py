"""MI355X-native CKKS hybrid key-switching (ModUp / KSKInnerProd / ModDown,
Rotate and hoisted HRotate) after de Castro et al., arXiv 2112.06396.

The compute path is the HIP library ``libhks.so`` (C ABI, ``include/hks.h``);
``paper_2112_06396_amd.hks`` is its thin ctypes binding.  Nothing is loaded at
import time, so ``paper_2112_06396_amd.synth`` can be imported without a GPU.
"""
