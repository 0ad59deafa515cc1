"""MI355X-native submatrix-method density matrix, P = 1/2 (I - sign(H - mu I)).

The compute path is libsmsign.so (HIP kernels for gfx950 behind a C ABI,
declared in include/smsign.h); `smsign` is its ctypes binding.  Importing the
package does not load the library; the first call does, and fails loudly if
it has not been built (`python -m paper_2205_14741_amd.build`).
"""
from . import smsign  # noqa: F401

__all__ = ["smsign"]
