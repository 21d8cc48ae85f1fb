"""MI355X-native hot path of PICCS-regularised Krylov CBCT reconstruction.

The compute path is the C-ABI HIP library ``libcbct.so`` built from ``csrc/``;
``paper_2509_08574_amd.cbct`` is its thin ctypes binding.  Importing the package
does not load the library.
"""
__all__ = ["cbct", "synth"]
