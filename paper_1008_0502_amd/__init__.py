"""MI355X-native saliency -> Kalman prior -> MRF weight path (arXiv:1008.0502).

The compute path is libsalprior.so (hand-written HIP kernels for gfx950 behind the
C-ABI of include/salprior.h).  Submodules: api (PyTorch binding), synth (seeded
synthetic clips), build (hipcc build of the library).
"""
from ._lib import LIB_PATH, SalpriorError, load  # noqa: F401

__all__ = ["LIB_PATH", "SalpriorError", "load"]
