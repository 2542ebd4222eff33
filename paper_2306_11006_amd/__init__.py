"""MI355X-native batched CGGI gate bootstrapping (ArctyrEX, arXiv 2306.11006).

The compute path is the C-ABI library ``libcggi.so`` (hand-written HIP for
gfx950, declared in ``include/cggi.h``); ``paper_2306_11006_amd.cggi`` is
its thin ctypes binding.  ``params`` and ``inputs`` hold parameter sets and
seeded synthetic inputs.
"""
