"""MI355X-native Whitted ray tracer (arXiv 1504.03151 hot path).

The tracer itself is the HIP library ``libmirt.so`` behind the C-ABI declared
in ``include/mirt.h``; ``paper_1504_03151_amd.rt`` is its thin Python binding.
``scenes`` generates seeded synthetic inputs.
"""
