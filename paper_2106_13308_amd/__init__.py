"""MI355X-native hot path of autoregressive-model VQMC for diagonal Ising / Max-Cut.

The compute path is the C-ABI library ``libvqmc.so`` (hand-written HIP kernels for
gfx950); :mod:`paper_2106_13308_amd.binding` marshals torch tensors into it.  Importing
this package loads nothing native; the binding loads the library on first use and
raises if it has not been built.
"""
__version__ = "0.1.0"
