"""MI355X-native pencil 3D FFT (the single-GPU hot path of DaggerFFT).

``paper_2601_12209_amd.fft3d`` is the torch-facing binding of the C ABI in
``include/fft3d.h``; the kernels live in ``csrc/`` and are built into
``libfft3d.so`` by ``paper_2601_12209_amd.build``.
"""
