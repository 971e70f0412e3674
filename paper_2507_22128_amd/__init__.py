"""MI355X-native major-cycle imager (arXiv 2507.22128 hot path).

``paper_2507_22128_amd.imager`` is the ctypes binding of ``libimager.so``
(HIP kernels for gfx950 behind the C-ABI declared in ``include/imager.h``);
``paper_2507_22128_amd.synth`` generates seeded synthetic workloads.
Nothing is loaded at import time.
"""
