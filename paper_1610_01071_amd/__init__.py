"""MI355X-native hot path of wavelet-based equation-free projective integration
for 1D1V electrostatic PIC (Cazeaux & Hesthaven, arXiv:1610.01071).

The compute lives in libefpi.so (HIP kernels for gfx950 behind the C ABI of
include/efpi.h); :mod:`paper_1610_01071_amd.efpi` is its Python binding.
"""
