"""MI355X-native beyond-Limber 3x2pt C_ell (the Blast method, arXiv:2410.03632).

The compute path lives in the HIP library built from ``csrc/`` and is reached
through ``paper_2410_03632_amd.blast`` (ctypes binding).  ``workloads`` holds the
seeded synthetic inputs.  Importing the package itself loads nothing native.
"""
__all__ = ["workloads", "blast"]
