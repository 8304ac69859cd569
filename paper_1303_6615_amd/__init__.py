"""MI355X-native asymptotic parareal for the 1D rotating shallow water system.

The compute path is the HIP library built from csrc/ (loaded on first use by
paper_1303_6615_amd.binding); importing this package loads nothing.
"""
__all__ = ["inputs", "binding"]
