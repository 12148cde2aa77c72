"""Time-domain Lienard-Wiechert radiation spectra on MI355X (gfx950).

The hot path -- arrival time and field of every (particle, step, pixel)
triple, the linear-interpolation deposit onto each pixel's uniform observer
grid, and the FFT to |E(w)|^2, plus the direct frequency-domain sum and the
adjoints -- runs in hand-written HIP kernels behind the C ABI of
``include/lw.h`` (``liblw.so``).  ``lw`` is the thin ctypes binding; importing
this package does not load the library (``lw.load()`` does, and fails loudly if
it is missing).
"""
__all__ = ["inputs", "grid", "lw"]
