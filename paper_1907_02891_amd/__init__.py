"""MI355X-native FFT evaluation of artificial night-sky-brightness maps.

The map of artificial sky brightness is the 2-D linear convolution of a
projected ground-radiance grid with a shift-invariant point-spread matrix
(Bara et al. 2019, Sec. 2.3, Eq. 7), evaluated through the convolution
theorem (Eq. 9) with zero-padded transforms (Sec. 2.5).  The transforms,
the spectrum multiply and the crop run in hand-written HIP kernels for gfx950
behind the C ABI declared in include/lp.h; `lp` is its Python binding.

Importing this package loads nothing; `paper_1907_02891_amd.lp` loads the
shared library and raises if it is missing.
"""
__all__ = ["lp", "synth"]
