"""MI355X-native explicit 3-D diffusion step with implicit-global-grid halo
updates (Omlin, Raess, Utkin, arXiv 2211.15716), behind a C-ABI HIP library.

Importing the package loads nothing; the HIP library is loaded on first use
by ``paper_2211_15716_amd.igg`` and raises if it is missing.
"""
__all__ = ["igg", "diffusion", "synth"]
