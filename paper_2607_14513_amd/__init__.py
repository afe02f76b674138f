"""MI355X-native BC1/BC7 coding of 3D Gaussian Splatting SH colour.

Implements the data-parallel path of Said & Rauwendaal, "Compression of 3D
Gaussian Splatting Data Using GPU-friendly Graphics Texture Coding": colour /
space reorder, 16 primitives per 4x4 band block, BC1/BC7 encoding with a
per-band rate choice, and random-access decode + SH evaluation -- all in HIP
kernels for gfx950 behind the C ABI of include/gsbc.h.

    from paper_2607_14513_amd import gsbc      # ctypes binding (needs libgsbc.so)
    from paper_2607_14513_amd import synth     # seeded synthetic inputs
"""
__all__ = ["gsbc", "synth"]
