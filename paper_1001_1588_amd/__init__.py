"""FFT EnKF analysis step on AMD Instinct MI355X (gfx950).

``analyze(ens, data, R_spec, seed)`` runs one analysis of the FFT Ensemble
Kalman Filter (Mandel, Beezley and Kondratenko, Section 2.1, eq. (2) and (3))
through the hand-written HIP kernels of libfftenkf.so; see include/fftenkf.h.
The binding is imported lazily so that the input generator (``twin``) can be
used without a GPU.
"""

__all__ = ["analyze", "debug_spectra", "debug_perturb", "workspace_bytes", "max_members", "twin"]


def __getattr__(name):
    if name in ("analyze", "debug_spectra", "debug_perturb", "workspace_bytes", "max_members", "lib"):
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError(name)
