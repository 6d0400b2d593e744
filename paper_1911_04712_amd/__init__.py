"""MI355X-native DPD solvent hot path (cell binning, DPD pair force, fused
velocity-Verlet) behind a C-ABI library; see include/dpd.h.

The GPU library is loaded lazily by `paper_1911_04712_amd.dpd`; importing
the package itself loads nothing.
"""
__all__ = ["inputs", "dpd"]
