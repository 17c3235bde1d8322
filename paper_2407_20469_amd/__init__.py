"""MI355X-native per-tile closed-form APIC reconstruction (arXiv 2407.20469).

The reconstruction runs in hand-written HIP kernels for gfx950 behind the C ABI
of include/apic.h (libapic.so, built in-tree by ``paper_2407_20469_amd.build``).
``paper_2407_20469_amd.apic`` is the ctypes binding.
"""

from . import apic  # noqa: F401
