"""MI355X-native Cahn-Hilliard update of the phase-field method of
Liu, Ng, Chong, Lohse & Verzicco (arXiv 2105.01865).

The compute path is the C-ABI library ``libch.so`` (HIP kernels for gfx950,
declared in ``include/ch.h``); ``paper_2105_01865_amd.ch`` is its thin
Python binding.  ``paper_2105_01865_amd.inputs`` builds seeded synthetic
inputs.  Importing the package does not load the GPU library.
"""
__all__ = ["ch", "inputs"]
