"""MI355X-native Tau1 lattice Boltzmann stream-and-collide (gfx950, HIP).

The compute path is the C-ABI library ``libtau1.so`` built from ``csrc/``;
:mod:`paper_2312_14742_amd.tau1` is a thin ctypes binding over it.  Importing
this package does not load the library; the binding loads it on first use and
raises if it is missing.
"""
__all__ = ["tau1", "inputs"]
