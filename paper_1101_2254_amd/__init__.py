"""MI355X-native hot path of GPU galaxy fitting (Barsdell, Barnes & Fluke,
"Fitting Galaxies on GPUs"): Sersic model evaluation, PSF convolution and
chi^2 (steps 1-3 of the fitting loop), their derivatives and a device-resident
Levenberg-Marquardt driver, as hand-written HIP kernels for gfx950 behind the
C ABI of ``include/gf.h``.

``paper_1101_2254_amd.ops`` is the tensor-level API; ``paper_1101_2254_amd._lib``
the raw binding; ``paper_1101_2254_amd.build`` compiles ``libgf.so``.
Importing the package does not load the library or touch the GPU.
"""
__all__ = ["ops", "build"]
