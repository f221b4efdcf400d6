"""MI355X-native 2D TM FDTD forward / adjoint / eps_r-sigma gradient library
(GPR dual-parameter full-waveform inversion hot path, arXiv 2506.20513).

The compute path is the HIP library ``libfwi.so`` (built from ``csrc/``)
behind the C ABI declared in ``include/fwi.h``; ``fwi`` is its thin ctypes
binding.  ``inputs`` holds the seeded synthetic input generators.
"""
